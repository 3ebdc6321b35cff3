// Training-set evaluation for the separable natural evolution strategy on
// gfx950 (paper, Sec. II E): the loss of a whole population of parameter
// vectors over many small periodic structures, and the SNES sampling and
// update steps.
//
// Structures are concatenated into one system (as the paper does, Sec. II F)
// with a cell per structure.  Their neighbour lists are built once, when the
// dataset is created.  One launch of the partial-force kernel evaluates every
// (atom, individual) pair; a population gather turns the partials into per-
// atom loss terms; float64 sums over each structure and then over structures
// give the loss components of each individual, in a fixed order.
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <atomic>

#include "nep_device.h"

namespace nep {
namespace {

inline unsigned blocks_for(size_t work, int block) { return (unsigned)((work + block - 1) / block); }

constexpr int kLanes = 4;  // lanes per atom in the population gather (as in pass 1)

// ------------------------------------------------------- dataset lists

// Wrap every position into its structure's cell; record the integer offsets
// that remain after rounding (normally zero).
__global__ void k_ds_wrap(int N, double* __restrict__ pos, const double* __restrict__ boxes,
                          const double* __restrict__ boxinv, const int* __restrict__ struct_of,
                          int* __restrict__ wrap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double* H = boxes + 9 * (size_t)struct_of[i];
  const double* Hi = boxinv + 9 * (size_t)struct_of[i];
  double r[3] = {pos[i], pos[N + i], pos[2 * N + i]};
  int w[3];
  for (int a = 0; a < 3; ++a) w[a] = (int)floor(r[0] * Hi[a] + r[1] * Hi[3 + a] + r[2] * Hi[6 + a]);
  for (int c = 0; c < 3; ++c) {
    r[c] -= ((double)w[0] * H[c] + (double)w[1] * H[3 + c]) + (double)w[2] * H[6 + c];
    pos[c * N + i] = r[c];
  }
  for (int a = 0; a < 3; ++a)
    wrap[a * N + i] = (int)floor(r[0] * Hi[a] + r[1] * Hi[3 + a] + r[2] * Hi[6 + a]);
}

// One wave per atom: every atom j of the same structure and every image m in
// [-K, K]^3 of the wrapped frame, numbered in (j, m0, m1, m2) order; 64 such
// candidates are tested at a time and a ballot keeps the serial order.  The
// angular-range entries come first (first pass), then the rest.
__global__ __launch_bounds__(256) void k_ds_build(
    int N, int cap, const double* __restrict__ pos, const double* __restrict__ boxes,
    const int* __restrict__ struct_of, const int* __restrict__ off, const int* __restrict__ kimg,
    const int* __restrict__ wrap, double rc2_r, double rc2_a, uint32_t* __restrict__ nl,
    int* __restrict__ cnt_r, int* __restrict__ cnt_a, int* __restrict__ flags) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gid / 64;
  const int k = gid % 64;
  if (i >= N) return;  // whole waves leave together
  const unsigned long long below = (1ull << k) - 1ull;
  const int s = struct_of[i];
  const double* H = boxes + 9 * (size_t)s;
  const int j0 = off[s], nj = off[s + 1] - off[s];
  const int K0 = kimg[3 * s], K1 = kimg[3 * s + 1], K2 = kimg[3 * s + 2];
  const int w1n = 2 * K1 + 1, w2n = 2 * K2 + 1;
  const int nimg = (2 * K0 + 1) * w1n * w2n;
  const int total = nj * nimg;
  const double xi = pos[i], yi = pos[N + i], zi = pos[2 * N + i];
  const int wi0 = wrap[i], wi1 = wrap[N + i], wi2 = wrap[2 * N + i];
  int count = 0;
  bool overflow = false, bad_image = false;
  for (int pass = 0; pass < 2; ++pass) {
    for (int base = 0; base < total; base += 64) {
      const int c = base + k;
      bool keep = false;
      uint32_t entry = 0;
      if (c < total) {
        const int j = j0 + c / nimg;
        const int mi = c % nimg;
        const int m0 = mi / (w1n * w2n) - K0;
        const int m1 = (mi / w2n) % w1n - K1;
        const int m2 = mi % w2n - K2;
        const int n0 = m0 + wi0 - wrap[j], n1 = m1 + wi1 - wrap[N + j], n2 = m2 + wi2 - wrap[2 * N + j];
        if (!(j == i && n0 == 0 && n1 == 0 && n2 == 0)) {
          const double r2 =
              list_r2(pos[j], pos[N + j], pos[2 * N + j], xi, yi, zi, n0, n1, n2, H);
          const bool in_a = r2 < rc2_a;
          keep = pass == 0 ? in_a : (!in_a && r2 < rc2_r);
          if (keep && (n0 < -3 || n0 > 3 || n1 < -3 || n1 > 3 || n2 < -3 || n2 > 3)) {
            bad_image = true;
            keep = false;
          }
          entry = pack_entry(j, n0, n1, n2);
        }
      }
      const unsigned long long ball = __ballot(keep);
      if (keep) {
        const int slot = count + __popcll(ball & below);
        if (slot < cap)
          nl[(size_t)slot * N + i] = entry;
        else
          overflow = true;
      }
      count += __popcll(ball);
    }
    if (pass == 0 && k == 0) cnt_a[i] = min(count, cap);
  }
  if (k == 0) cnt_r[i] = min(count, cap);
  if (overflow) flags[kFlagOverflow] = 1;
  if (bad_image) flags[kFlagImage] = 1;
}

// ------------------------------------------------- population loss terms

// One individual: per atom F_i = sum_j p_ij - sum_j p_ji into F_out [3][N],
// and the terms (U_i, W_i row-major 9, W_i = sum_j r_ij (x) p_ji) at
// terms[q N + i].
template <int L>
__global__ __launch_bounds__(kBlock) void k_ds_gather(
    int N, const double* __restrict__ pos, const double* __restrict__ boxes,
    const int* __restrict__ struct_of, const uint32_t* __restrict__ nl,
    const int* __restrict__ cnt_r, const Partial3* __restrict__ pin, const float* __restrict__ fown,
    const float* __restrict__ U, double* __restrict__ terms, float* __restrict__ F_out) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gid / L;
  const int lane = gid % L;
  const bool active = i < N;
  const int ii = active ? i : 0;
  const int cr = active ? cnt_r[i] : 0;
  const double xi = pos[ii], yi = pos[N + ii], zi = pos[2 * N + ii];
  const double* H = boxes + 9 * (size_t)struct_of[ii];
  float f0 = 0.f, f1 = 0.f, f2 = 0.f;
  float w[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) w[q] = 0.f;
  for (int s = lane; s < cr; s += L) {
    const size_t idx = (size_t)s * N + i;
    int j;
    float dx, dy, dz;
    displacement(nl[idx], pos, N, xi, yi, zi, H, j, dx, dy, dz);
    const Partial3 pji = pin[idx];
    f0 -= pji.x;
    f1 -= pji.y;
    f2 -= pji.z;
    w[0] += dx * pji.x;
    w[1] += dx * pji.y;
    w[2] += dx * pji.z;
    w[3] += dy * pji.x;
    w[4] += dy * pji.y;
    w[5] += dy * pji.z;
    w[6] += dz * pji.x;
    w[7] += dz * pji.y;
    w[8] += dz * pji.z;
  }
  f0 = group_sum<L>(f0);
  f1 = group_sum<L>(f1);
  f2 = group_sum<L>(f2);
#pragma unroll
  for (int q = 0; q < 9; ++q) w[q] = group_sum<L>(w[q]);
  if (active && lane == 0) {
    F_out[i] = f0 + fown[i];
    F_out[N + i] = f1 + fown[N + i];
    F_out[2 * N + i] = f2 + fown[2 * N + i];
    terms[i] = (double)U[i];
#pragma unroll
    for (int q = 0; q < 9; ++q) terms[(size_t)(1 + q) * N + i] = (double)w[q];
  }
}

// Per structure s = blockIdx.x: energy[s] = sum U_i and, unless NULL,
// virial[s][9] = sum W_i over the structure's atoms (forward terms layout).
__global__ __launch_bounds__(kBlock) void k_ds_totals(int N, const int* __restrict__ off,
                                                      const double* __restrict__ terms,
                                                      double* __restrict__ energy,
                                                      double* __restrict__ virial) {
  __shared__ double sw[kBlock / 64][10];
  const int s = blockIdx.x;
  double acc[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  for (int a = off[s] + threadIdx.x; a < off[s + 1]; a += blockDim.x)
#pragma unroll
    for (int q = 0; q < 10; ++q) acc[q] += terms[(size_t)q * N + a];
  const double v = block_sum<10>(acc, sw);
  if (threadIdx.x == 0) energy[s] = v;
  if (virial && threadIdx.x >= 1 && threadIdx.x < 10) virial[9 * (size_t)s + threadIdx.x - 1] = v;
}

// Per individual k = blockIdx.x: loss[k][6] = (L, L_e, L_f, L_v, L_1, L_2).
__global__ __launch_bounds__(kBlock) void k_ds_loss(int S, int N, int n_virial, int n_par,
                                                    const double* __restrict__ sq,
                                                    const float* __restrict__ Z, double le,
                                                    double lf, double lv, double l1, double l2,
                                                    double* __restrict__ loss) {
  __shared__ double sw[kBlock / 64][5];
  __shared__ double tot[5];
  const size_t pk = blockIdx.x;
  const double* q = sq + pk * 3 * (size_t)S;
  const float* z = Z + pk * (size_t)n_par;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int s = threadIdx.x; s < S; s += blockDim.x) {
    acc[0] += q[3 * s];
    acc[1] += q[3 * s + 1];
    acc[2] += q[3 * s + 2];
  }
  for (int v = threadIdx.x; v < n_par; v += blockDim.x) {
    const double x = (double)z[v];
    acc[3] += fabs(x);
    acc[4] += x * x;
  }
  const double v = block_sum<5>(acc, sw);
  if (threadIdx.x < 5) tot[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double Le = sqrt(tot[0] / S);
    const double Lf = sqrt(tot[1] / (3.0 * N));
    const double Lv = n_virial > 0 ? sqrt(tot[2] / (6.0 * n_virial)) : 0.0;
    const double L1 = tot[3] / n_par;
    const double L2 = sqrt(tot[4] / n_par);
    double* o = loss + 6 * pk;
    o[0] = le * Le + lf * Lf + lv * Lv + l1 * L1 + l2 * L2;
    o[1] = Le;
    o[2] = Lf;
    o[3] = Lv;
    o[4] = L1;
    o[5] = L2;
  }
}

// ------------------------------------------------------- SNES steps

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each round
// multiplies words 0 and 2 by 0xD2511F53 and 0xCD9E8D57, mixes the high
// halves with words 1 and 3 and the key; the key advances by 0x9E3779B9 and
// 0xBB67AE85 between rounds.
__device__ __forceinline__ void philox(uint32_t (&x)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t a = (uint64_t)0xD2511F53u * x[0];
    const uint64_t b = (uint64_t)0xCD9E8D57u * x[2];
    const uint32_t n0 = (uint32_t)(b >> 32) ^ x[1] ^ k0;
    const uint32_t n2 = (uint32_t)(a >> 32) ^ x[3] ^ k1;
    x[0] = n0;
    x[1] = (uint32_t)b;
    x[2] = n2;
    x[3] = (uint32_t)a;
  }
}

// Generation `gen`, or gen_dev[0] when gen_dev is not NULL.
__global__ void k_snes_sample(int n_par, const float* __restrict__ m, const float* __restrict__ s,
                              uint32_t key0, uint32_t key1, uint32_t gen,
                              const int* __restrict__ gen_dev, float* __restrict__ r,
                              float* __restrict__ Z) {
#pragma clang fp contract(off)
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (4 * b >= n_par) return;
  if (gen_dev) gen = (uint32_t)gen_dev[0];
  uint32_t x[4] = {(uint32_t)b, (uint32_t)k, gen, 0u};
  philox(x, key0, key1);
  double u[4];
  for (int t = 0; t < 4; ++t) u[t] = ((double)x[t] + 0.5) * (1.0 / 4294967296.0);
  const double twopi = 6.28318530717958647692;
  const double rad0 = sqrt(-2.0 * log(u[0])), rad1 = sqrt(-2.0 * log(u[2]));
  const double nrm[4] = {rad0 * cos(twopi * u[1]), rad0 * sin(twopi * u[1]),
                         rad1 * cos(twopi * u[3]), rad1 * sin(twopi * u[3])};
  for (int t = 0; t < 4; ++t) {
    const int v = 4 * b + t;
    if (v >= n_par) break;
    const float rv = (float)nrm[t];
    r[(size_t)k * n_par + v] = rv;
    Z[(size_t)k * n_par + v] = (float)((double)m[v] + (double)s[v] * (double)rv);
  }
}

// Every block ranks the population itself (P <= 1024), then updates its
// share of the parameters.
__global__ __launch_bounds__(kBlock) void k_snes_update(int n_par, int n_pop, float* __restrict__ m,
                                                        float* __restrict__ s,
                                                        const float* __restrict__ r,
                                                        const double* __restrict__ loss,
                                                        double eta_m, double eta_s) {
#pragma clang fp contract(off)
  __shared__ int order[1024];
  __shared__ double util[1024];
  __shared__ double key[1024];
  __shared__ double tot_s;
  // sort keys (NaN ranks last) and the unnormalised utilities of ranks 1..P
  const double top = log(n_pop / 2.0 + 1.0);
  for (int k = threadIdx.x; k < n_pop; k += blockDim.x) {
    const double lk = loss[6 * k];
    key[k] = lk != lk ? INFINITY : lk;
    const double v = top - log((double)(k + 1));
    util[k] = v > 0.0 ? v : 0.0;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n_pop; k += blockDim.x) {
    const double kk = key[k];
    int rank = 0;
    for (int j = 0; j < n_pop; ++j) {
      const double kj = key[j];
      rank += (kj < kk || (kj == kk && j < k)) ? 1 : 0;
    }
    order[rank] = k;
  }
  if (threadIdx.x == 0) {  // the normalising sum in rank order
    double tot = 0.0;
    for (int k = 0; k < n_pop; ++k) tot += util[k];
    tot_s = tot;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n_pop; k += blockDim.x) util[k] = util[k] / tot_s - 1.0 / n_pop;
  __syncthreads();
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_par) return;
  double gm = 0.0, gs = 0.0;
  // (unrolled so that the loads of several ranks are in flight together; the
  // sums keep rank order)
#pragma unroll 8
  for (int rank = 0; rank < n_pop; ++rank) {
    const double rv = (double)r[(size_t)order[rank] * n_par + v];
    gm += util[rank] * rv;
    gs += util[rank] * (rv * rv - 1.0);
  }
  const double sv = (double)s[v];
  m[v] = (float)((double)m[v] + eta_m * sv * gm);
  s[v] = (float)(sv * exp(0.5 * eta_s * gs));
}

// One wave: best[(g - g0) 6 + q] = loss terms of the best individual of
// generation g = counter[0] (NaN ranks last, ties by index), g0 = counter[1];
// then counter[0] = g + 1.
__global__ __launch_bounds__(64) void k_snes_record(int n_pop, const double* __restrict__ loss,
                                                    int* __restrict__ counter,
                                                    double* __restrict__ best) {
  if (blockIdx.x != 0) return;
  const int l = threadIdx.x;
  const int g = counter[0];
  if (best) {
    // lane minima over k = l, l + 64, ..., then the wave's (loss, index) minimum
    double lb = INFINITY;
    int b = n_pop;
    for (int k = l; k < n_pop; k += 64) {
      const double lk = loss[6 * k] != loss[6 * k] ? INFINITY : loss[6 * k];
      if (lk < lb || (lk == lb && k < b)) {
        lb = lk;
        b = k;
      }
    }
    for (int d = 32; d > 0; d >>= 1) {
      const double lo = __shfl_xor(lb, d, 64);
      const int bo = __shfl_xor(b, d, 64);
      if (lo < lb || (lo == lb && bo < b)) {
        lb = lo;
        b = bo;
      }
    }
    if (b >= n_pop) b = 0;  // every loss NaN: the first individual
    if (l < 6) best[(size_t)(g - counter[1]) * 6 + l] = loss[6 * b + l];
  }
  __syncthreads();  // every lane has read the counter
  if (l == 0) counter[0] = g + 1;
}

__global__ void k_set_counter(int* __restrict__ counter, int g) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    counter[0] = g;
    counter[1] = g;
  }
}

void invert_box(const double* H, double* Hi) {
  const double a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7],
               k = H[8];
  const double det = a * (e * k - f * h) - b * (d * k - f * g) + c * (d * h - e * g);
  Hi[0] = (e * k - f * h) / det;
  Hi[1] = (c * h - b * k) / det;
  Hi[2] = (b * f - c * e) / det;
  Hi[3] = (f * g - d * k) / det;
  Hi[4] = (a * k - c * g) / det;
  Hi[5] = (c * d - a * f) / det;
  Hi[6] = (d * h - e * g) / det;
  Hi[7] = (b * g - a * h) / det;
  Hi[8] = (a * e - b * d) / det;
}

// Wrap the dataset's positions and build its lists and reverse slots.
hipError_t build_dataset_lists(nep_ctx ctx, nep_dataset ds) {
  const int N = ds->N;
  hipStream_t st = ctx->stream;
  k_ds_wrap<<<blocks_for(N, kBlock), kBlock, 0, st>>>(N, ds->pos.ptr, ds->boxes.ptr,
                                                      ds->boxinv.ptr, ds->struct_of.ptr,
                                                      ds->wrap.ptr);
  k_ds_build<<<blocks_for((size_t)N * 64, 256), 256, 0, st>>>(
      N, ds->cap, ds->pos.ptr, ds->boxes.ptr, ds->struct_of.ptr, ds->off.ptr, ds->kimg.ptr,
      ds->wrap.ptr, ds->rc_r * ds->rc_r, ds->rc_a * ds->rc_a, ds->nl.ptr, ds->cnt_r.ptr,
      ds->cnt_a.ptr, ctx->flags.ptr);
  launch_reverse(ctx, N, ds->cap, ds->nl.ptr, ds->cnt_r.ptr, ds->cnt_a.ptr, ds->rev.ptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return prepare_dataset_geometry(ctx, ds);
}

nep_status check_dataset(nep_ctx ctx, nep_dataset ds) {
  if (!ds || ds->ctx != ctx) return fail(ctx, NEP_EINVAL, "dataset belongs to another context");
  if (!ctx->have_params) return fail(ctx, NEP_ESTATE, "nep_load_params must come first");
  if (!have_training_variant(ctx->hyper))
    return fail(ctx, NEP_ENOTIMPL, "dataset kernels are compiled for (8, 4, 4, 30) only");
  if (ds->rc_r != ctx->hyper.rc_radial || ds->rc_a != ctx->hyper.rc_angular)
    return fail(ctx, NEP_ESTATE, "dataset lists were built for other cutoffs");
  return NEP_OK;
}

// Workspace of snes_eval_population for n_pop individuals: dU/dq (32 floats
// per atom and individual), site energies and per-structure squared errors.
hipError_t ensure_population(nep_dataset ds, int n_pop) {
  const int N = ds->N, S = ds->S;
  hipError_t e = ds->dq.ensure((size_t)n_pop * N * 32);
  if (e == hipSuccess) e = ds->dqbound.ensure((size_t)n_pop);
  if (e == hipSuccess) e = ds->wfrag.ensure((size_t)n_pop * 12 * 64);
  if (e == hipSuccess) e = ds->wb2.ensure((size_t)n_pop);
  if (e == hipSuccess) e = ds->U.ensure((size_t)n_pop * N);
  if (e == hipSuccess) e = ds->struct_sq.ensure((size_t)n_pop * 3 * S);
  return e;
}

// Enqueue one population evaluation and its loss reduction.
hipError_t enqueue_population_loss(nep_ctx ctx, nep_dataset ds, int n_pop, const float* Z_dev,
                                   const double* lambda, double* loss_dev, int variant) {
  hipError_t r = launch_population(ctx, ds, n_pop, Z_dev, variant, true);
  if (r != hipSuccess) return r;
  launch_kernel(ctx, false, true, k_ds_loss, dim3(n_pop), dim3(kBlock), ds->S, ds->N,
                ds->n_virial, ctx->n_par, (const double*)ds->struct_sq.ptr, Z_dev, lambda[0],
                lambda[1], lambda[2], lambda[3], lambda[4], loss_dev);
  return hipGetLastError();
}

bool population_fits(nep_dataset ds) {
  return ds->tile_max <= population_max_structure() &&
         (size_t)ds->N * 32 * 65535 < (1ull << 62);
}

}  // namespace
}  // namespace nep

using namespace nep;

extern "C" {

nep_status nep_dataset_create(nep_ctx ctx, int n_struct, const int* n_atoms_host,
                              const double* boxes_host, const double* pos_host,
                              const double* energy_host, const double* forces_host,
                              const double* virial_host, const unsigned char* has_virial_host,
                              int max_neighbors, nep_dataset* out) {
  if (!ctx || !out) return NEP_EINVAL;
  *out = nullptr;
  if (!ctx->have_params) return fail(ctx, NEP_ESTATE, "nep_load_params must come first");
  if (!have_training_variant(ctx->hyper))
    return fail(ctx, NEP_ENOTIMPL, "dataset kernels are compiled for (8, 4, 4, 30) only");
  if (n_struct < 1) return fail(ctx, NEP_EINVAL, "n_struct must be >= 1");
  if (!n_atoms_host || !boxes_host || !pos_host || !energy_host || !forces_host || !virial_host ||
      !has_virial_host)
    return fail(ctx, NEP_EINVAL, "a host array is NULL");
  if (max_neighbors < 1) return fail(ctx, NEP_EINVAL, "max_neighbors must be >= 1");
  long long total = 0;
  for (int s = 0; s < n_struct; ++s) {
    if (n_atoms_host[s] < 1) return fail(ctx, NEP_EINVAL, "every structure needs >= 1 atom");
    total += n_atoms_host[s];
  }
  if (total > kMaxAtoms) return fail(ctx, NEP_EINVAL, "more than 2^23 - 1 atoms in total");
  if ((unsigned long long)total * (unsigned long long)max_neighbors >= (1ull << 31))
    return fail(ctx, NEP_EINVAL, "max_neighbors * total atoms must be below 2^31");
  const int N = (int)total, S = n_struct;
  const double rc_r = ctx->hyper.rc_radial, rc_a = ctx->hyper.rc_angular;
  std::vector<double> hinv((size_t)9 * S);
  std::vector<int> kimg((size_t)3 * S), off((size_t)S + 1), sof(N);
  std::vector<double> posT((size_t)3 * N), ftT((size_t)3 * N);
  std::vector<int> hv(S);
  int n_virial = 0;
  off[0] = 0;
  for (int s = 0; s < S; ++s) {
    const double* H = boxes_host + 9 * (size_t)s;
    for (int q = 0; q < 9; ++q)
      if (!std::isfinite(H[q])) return fail(ctx, NEP_EINVAL, "box has non-finite entries");
    invert_box(H, &hinv[9 * (size_t)s]);
    System probe;
    prepare_system_geometry(probe, H, rc_r, rc_a, 0.0);
    for (int a = 0; a < 3; ++a) {
      kimg[3 * s + a] = probe.kimg[a];
      if (probe.kimg[a] > 2 || !std::isfinite(hinv[9 * (size_t)s]))
        return fail(ctx, NEP_EINVAL,
                    "structure " + std::to_string(s) + ": cell thinner than half the cutoff");
    }
    off[s + 1] = off[s] + n_atoms_host[s];
    for (int a = off[s]; a < off[s + 1]; ++a) sof[a] = s;
    hv[s] = has_virial_host[s] ? 1 : 0;
    n_virial += hv[s];
  }
  for (int a = 0; a < N; ++a)
    for (int c = 0; c < 3; ++c) {
      posT[(size_t)c * N + a] = pos_host[3 * (size_t)a + c];
      ftT[(size_t)c * N + a] = forces_host[3 * (size_t)a + c];
    }
  nep_dataset ds = new (std::nothrow) nep_dataset_s();
  if (!ds) return fail(ctx, NEP_ENOMEM, "dataset");
  static std::atomic<unsigned long long> next_serial{0};
  ds->serial = ++next_serial;
  ds->ctx = ctx;
  ds->S = S;
  ds->N = N;
  ds->cap = max_neighbors;
  ds->n_virial = n_virial;
  ds->rc_r = rc_r;
  ds->rc_a = rc_a;
  ds->off_host = off;
  DeviceGuard guard(ctx->device);
  hipError_t e = hipSuccess;
  const size_t ncap = (size_t)N * max_neighbors;
  if (e == hipSuccess) e = ds->pos.ensure((size_t)3 * N);
  if (e == hipSuccess) e = ds->boxes.ensure((size_t)9 * S);
  if (e == hipSuccess) e = ds->boxinv.ensure((size_t)9 * S);
  if (e == hipSuccess) e = ds->struct_of.ensure(N);
  if (e == hipSuccess) e = ds->off.ensure((size_t)S + 1);
  if (e == hipSuccess) e = ds->kimg.ensure((size_t)3 * S);
  if (e == hipSuccess) e = ds->e_tar.ensure(S);
  if (e == hipSuccess) e = ds->f_tar.ensure((size_t)3 * N);
  if (e == hipSuccess) e = ds->w_tar.ensure((size_t)6 * S);
  if (e == hipSuccess) e = ds->has_v.ensure(S);
  if (e == hipSuccess) e = ds->nl.ensure(ncap);
  if (e == hipSuccess) e = ds->rev.ensure(ncap);
  if (e == hipSuccess) e = ds->cnt_r.ensure(N);
  if (e == hipSuccess) e = ds->cnt_a.ensure(N);
  if (e == hipSuccess) e = ds->wrap.ensure((size_t)3 * N);
  hipStream_t st = ctx->stream;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  up(ds->pos.ptr, posT.data(), sizeof(double) * 3 * N);
  up(ds->boxes.ptr, boxes_host, sizeof(double) * 9 * S);
  up(ds->boxinv.ptr, hinv.data(), sizeof(double) * 9 * S);
  up(ds->struct_of.ptr, sof.data(), sizeof(int) * N);
  up(ds->off.ptr, off.data(), sizeof(int) * (S + 1));
  up(ds->kimg.ptr, kimg.data(), sizeof(int) * 3 * S);
  up(ds->e_tar.ptr, energy_host, sizeof(double) * S);
  up(ds->f_tar.ptr, ftT.data(), sizeof(double) * 3 * N);
  up(ds->w_tar.ptr, virial_host, sizeof(double) * 6 * S);
  up(ds->has_v.ptr, hv.data(), sizeof(int) * S);
  if (e == hipSuccess) e = build_dataset_lists(ctx, ds);
  if (e != hipSuccess) {
    nep_dataset_destroy(ds);
    return check_hip(ctx, e, "creating the dataset");
  }
  // the host buffers above are read by the copies: wait before returning
  nep_status stt = nep_synchronize(ctx);
  if (stt != NEP_OK) {
    nep_dataset_destroy(ds);
    return stt;
  }
  *out = ds;
  return NEP_OK;
}

nep_status nep_dataset_pairs(nep_dataset ds, long long* radial_pairs, long long* angular_pairs) {
  if (!ds || !radial_pairs || !angular_pairs) return NEP_EINVAL;
  *radial_pairs = ds->pairs_r;
  *angular_pairs = ds->pairs_a;
  return NEP_OK;
}

void nep_dataset_destroy(nep_dataset ds) {
  if (!ds) return;
  DeviceGuard guard(ds->ctx->device);
  (void)hipStreamSynchronize(ds->ctx->stream);
  ds->pos.release();
  ds->boxes.release();
  ds->boxinv.release();
  ds->struct_of.release();
  ds->off.release();
  ds->kimg.release();
  ds->e_tar.release();
  ds->f_tar.release();
  ds->w_tar.release();
  ds->has_v.release();
  ds->nl.release();
  ds->cnt_r.release();
  ds->cnt_a.release();
  ds->rev.release();
  ds->wrap.release();
  ds->pin.release();
  ds->fown.release();
  ds->U.release();
  ds->dq.release();
  ds->dqbound.release();
  ds->wfrag.release();
  ds->wb2.release();
  ds->atom_terms.release();
  ds->struct_sq.release();
  ds->grad_rec.release();
  ds->grad_part.release();
  ds->release_cache();
  delete ds;
}

nep_status nep_dataset_set_positions(nep_ctx ctx, nep_dataset ds, const double* pos_dev) {
  if (!ctx) return NEP_EINVAL;
  if (!ds || ds->ctx != ctx) return fail(ctx, NEP_EINVAL, "dataset belongs to another context");
  if (!pos_dev) return fail(ctx, NEP_EINVAL, "pos_dev is NULL");
  DeviceGuard guard(ctx->device);
  hipError_t e = hipMemcpyAsync(ds->pos.ptr, pos_dev, sizeof(double) * 3 * ds->N,
                                hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = build_dataset_lists(ctx, ds);
  if (e != hipSuccess) return check_hip(ctx, e, "rebuilding dataset lists");
  return nep_synchronize(ctx);
}

nep_status nep_dataset_get_positions(nep_ctx ctx, nep_dataset ds, double* pos_dev) {
  if (!ctx) return NEP_EINVAL;
  if (!ds || ds->ctx != ctx) return fail(ctx, NEP_EINVAL, "dataset belongs to another context");
  if (!pos_dev) return fail(ctx, NEP_EINVAL, "pos_dev is NULL");
  DeviceGuard guard(ctx->device);
  return check_hip(ctx,
                   hipMemcpyAsync(pos_dev, ds->pos.ptr, sizeof(double) * 3 * ds->N,
                                  hipMemcpyDeviceToDevice, ctx->stream),
                   "copying dataset positions");
}

nep_status nep_dataset_compute(nep_ctx ctx, nep_dataset ds, const float* z_dev,
                               double* energy_dev, float* forces_dev, double* virial_dev) {
  if (!ctx) return NEP_EINVAL;
  nep_status chk = check_dataset(ctx, ds);
  if (chk != NEP_OK) return chk;
  if (!z_dev || !energy_dev || !forces_dev) return fail(ctx, NEP_EINVAL, "NULL argument");
  const int N = ds->N, S = ds->S;
  DeviceGuard guard(ctx->device);
  hipError_t e = ds->pin.ensure((size_t)ds->cap * N);
  if (e == hipSuccess) e = ds->fown.ensure((size_t)3 * N);
  if (e == hipSuccess) e = ds->U.ensure((size_t)N);
  if (e == hipSuccess) e = ds->atom_terms.ensure((size_t)10 * N);
  if (e != hipSuccess) return check_hip(ctx, e, "allocating dataset workspace");
  e = timed(ctx, 0, [&] { return launch_partials_population(ctx, ds, 1, z_dev); });
  if (e == hipSuccess)
    e = timed(ctx, 1, [&] {
      launch_kernel(ctx, true, false, k_ds_gather<kLanes>,
                    dim3(blocks_for((size_t)N * kLanes, kBlock)), dim3(kBlock), N,
                    (const double*)ds->pos.ptr, (const double*)ds->boxes.ptr,
                    (const int*)ds->struct_of.ptr, (const uint32_t*)ds->nl.ptr,
                    (const int*)ds->cnt_r.ptr, (const Partial3*)ds->pin.ptr,
                    (const float*)ds->fown.ptr, (const float*)ds->U.ptr, ds->atom_terms.ptr,
                    forces_dev);
      launch_kernel(ctx, false, true, k_ds_totals, dim3(S), dim3(kBlock), N,
                    (const int*)ds->off.ptr, (const double*)ds->atom_terms.ptr, energy_dev,
                    virial_dev);
      return hipGetLastError();
    });
  return check_hip(ctx, e, "launching dataset forward");
}

nep_status nep_dataset_backward(nep_ctx ctx, nep_dataset ds, const float* z_dev,
                                const double* gE_dev, const float* gF_dev,
                                const float* forces_dev, double* grad_pos_dev,
                                double* grad_z_dev, float* grad_z32_dev) {
  if (!ctx) return NEP_EINVAL;
  nep_status chk = check_dataset(ctx, ds);
  if (chk != NEP_OK) return chk;
  if (!z_dev || !grad_z_dev) return fail(ctx, NEP_EINVAL, "z_dev and grad_z_dev are required");
  if (grad_pos_dev && !forces_dev)
    return fail(ctx, NEP_EINVAL, "grad_pos_dev needs forces_dev from nep_dataset_compute");
  DeviceGuard guard(ctx->device);
  hipError_t e = timed(ctx, 0, [&] {
    return launch_backward(ctx, ds, z_dev, gE_dev, gF_dev, forces_dev, grad_pos_dev, grad_z_dev,
                           grad_z32_dev);
  });
  return check_hip(ctx, e, "launching the backward pass");
}

nep_status snes_eval_population(nep_ctx ctx, nep_dataset ds, int n_pop, const float* Z_dev,
                                const double* lambda_host, double* loss_dev) {
  if (!ctx) return NEP_EINVAL;
  nep_status chk = check_dataset(ctx, ds);
  if (chk != NEP_OK) return chk;
  if (n_pop < 1 || n_pop > 65535) return fail(ctx, NEP_EINVAL, "n_pop must be in [1, 65535]");
  if (!Z_dev || !lambda_host || !loss_dev) return fail(ctx, NEP_EINVAL, "NULL argument");
  if (!population_fits(ds))
    return fail(ctx, NEP_EINVAL, "a structure has more atoms than the population kernels hold");
  DeviceGuard guard(ctx->device);
  hipError_t e = ensure_population(ds, n_pop);
  if (e != hipSuccess) return check_hip(ctx, e, "allocating population workspace");
  e = timed(ctx, 0, [&] {
    return enqueue_population_loss(ctx, ds, n_pop, Z_dev, lambda_host, loss_dev, ds->pop_variant);
  });
  return check_hip(ctx, e, "launching population kernels");
}

nep_status snes_sample(nep_ctx ctx, int n_par, int n_pop, const float* m_dev, const float* s_dev,
                       unsigned long long seed, int generation, float* r_dev, float* Z_dev) {
  if (!ctx) return NEP_EINVAL;
  if (n_par < 1 || n_pop < 1 || n_pop > 65535)
    return fail(ctx, NEP_EINVAL, "n_par >= 1 and 1 <= n_pop <= 65535 required");
  if (generation < 0) return fail(ctx, NEP_EINVAL, "generation must be >= 0");
  if (!m_dev || !s_dev || !r_dev || !Z_dev) return fail(ctx, NEP_EINVAL, "NULL argument");
  DeviceGuard guard(ctx->device);
  hipError_t e = hipSuccess;
  {
    const int nb = (n_par + 3) / 4;
    launch_kernel(ctx, true, true, k_snes_sample, dim3(blocks_for(nb, kBlock), n_pop),
                  dim3(kBlock), n_par, m_dev, s_dev, (uint32_t)(seed & 0xFFFFFFFFull),
                  (uint32_t)(seed >> 32), (uint32_t)generation, (const int*)nullptr, r_dev, Z_dev);
    e = hipGetLastError();
  }
  return check_hip(ctx, e, "launching the SNES sampler");
}

nep_status snes_update(nep_ctx ctx, int n_par, int n_pop, float* m_dev, float* s_dev,
                       const float* r_dev, const double* loss_dev, double eta_m, double eta_s) {
  if (!ctx) return NEP_EINVAL;
  if (n_par < 1 || n_pop < 1 || n_pop > 1024)
    return fail(ctx, NEP_EINVAL, "n_par >= 1 and 1 <= n_pop <= 1024 required");
  if (!m_dev || !s_dev || !r_dev || !loss_dev) return fail(ctx, NEP_EINVAL, "NULL argument");
  if (!(eta_m > 0.0)) eta_m = 1.0;
  if (!(eta_s > 0.0)) eta_s = (3.0 + std::log((double)n_par)) / (5.0 * std::sqrt((double)n_par));
  DeviceGuard guard(ctx->device);
  hipError_t e = hipSuccess;
  {
    launch_kernel(ctx, true, true, k_snes_update, dim3(blocks_for(n_par, kBlock)), dim3(kBlock),
                  n_par, n_pop, m_dev, s_dev, r_dev, loss_dev, eta_m, eta_s);
    e = hipGetLastError();
  }
  return check_hip(ctx, e, "launching the SNES update");
}

nep_status snes_autotune(nep_ctx ctx, nep_dataset ds, int n_pop, const float* Z_dev, int reps,
                         int* atoms_out, double* ms_out) {
  if (!ctx) return NEP_EINVAL;
  nep_status chk = check_dataset(ctx, ds);
  if (chk != NEP_OK) return chk;
  if (n_pop < 1 || n_pop > 65535) return fail(ctx, NEP_EINVAL, "n_pop must be in [1, 65535]");
  if (reps < 1 || reps > 1000) return fail(ctx, NEP_EINVAL, "reps must be in [1, 1000]");
  if (!Z_dev) return fail(ctx, NEP_EINVAL, "Z_dev is NULL");
  if (!population_fits(ds))
    return fail(ctx, NEP_EINVAL, "a structure has more atoms than the population kernels hold");
  DeviceGuard guard(ctx->device);
  hipError_t e = ensure_population(ds, n_pop);
  if (e != hipSuccess) return check_hip(ctx, e, "allocating population workspace");
  const bool timing = ctx->timer.on;
  ctx->timer.on = false;
  hipEvent_t a = nullptr, b = nullptr;
  e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  const int nv = population_variants();
  int best = ds->pop_variant;
  double best_ms = 0.0;
  for (int v = 0; v < nv && e == hipSuccess; ++v) {
    e = launch_population(ctx, ds, n_pop, Z_dev, v, true);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(a, ctx->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r)
      e = launch_population(ctx, ds, n_pop, Z_dev, v, true);
    if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    const double per = (double)ms / reps;
    if (ms_out) ms_out[v] = per;
    if (e == hipSuccess && (v == 0 || per < best_ms)) {
      best = v;
      best_ms = per;
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  ctx->timer.on = timing;
  if (e != hipSuccess) return check_hip(ctx, e, "timing population kernels");
  ds->pop_variant = best;
  ds->pop_tuned = true;
  if (atoms_out) *atoms_out = population_atoms(best);
  return nep_synchronize(ctx);
}

nep_status snes_set_tile(nep_ctx ctx, nep_dataset ds, int atoms) {
  if (!ctx) return NEP_EINVAL;
  if (!ds || ds->ctx != ctx) return fail(ctx, NEP_EINVAL, "dataset belongs to another context");
  for (int v = 0; v < population_variants(); ++v)
    if (population_atoms(v) == atoms) {
      ds->pop_variant = v;
      return NEP_OK;
    }
  return fail(ctx, NEP_EINVAL, "atoms must be 16, 32 or 64");
}

nep_status snes_run(nep_ctx ctx, nep_dataset ds, int n_par, int n_pop, float* m_dev,
                    float* s_dev, unsigned long long seed, int generation, int n_gen,
                    const double* lambda_host, double eta_m, double eta_s, float* r_dev,
                    float* Z_dev, double* loss_dev, double* best_dev) {
  if (!ctx) return NEP_EINVAL;
  nep_status chk = check_dataset(ctx, ds);
  if (chk != NEP_OK) return chk;
  if (n_par != ctx->n_par) return fail(ctx, NEP_EINVAL, "n_par differs from the loaded model");
  if (n_pop < 1 || n_pop > 1024) return fail(ctx, NEP_EINVAL, "n_pop must be in [1, 1024]");
  if (generation < 0 || n_gen < 0 || (long long)generation + n_gen > 2147483647LL)
    return fail(ctx, NEP_EINVAL, "generation range out of bounds");
  if (!m_dev || !s_dev || !r_dev || !Z_dev || !loss_dev || !lambda_host)
    return fail(ctx, NEP_EINVAL, "NULL argument");
  if (!population_fits(ds))
    return fail(ctx, NEP_EINVAL, "a structure has more atoms than the population kernels hold");
  if (n_gen == 0) return NEP_OK;
  if (!(eta_m > 0.0)) eta_m = 1.0;
  if (!(eta_s > 0.0)) eta_s = (3.0 + std::log((double)n_par)) / (5.0 * std::sqrt((double)n_par));
  DeviceGuard guard(ctx->device);
  hipError_t e = ensure_population(ds, n_pop);
  if (e == hipSuccess) e = ctx->gen_counter.ensure(2);
  if (e != hipSuccess) return check_hip(ctx, e, "allocating SNES workspace");
  SnesGraph& G = ctx->snes_graph;
  const std::vector<const void*> pk = {ds, m_dev, s_dev, r_dev, Z_dev, loss_dev, best_dev,
                                       ds->dq.ptr, ds->U.ptr, ds->struct_sq.ptr, ds->pfrag.ptr,
                                       ds->ppair.ptr, ds->qpad.ptr, ds->dqbound.ptr,
                                       ds->tbound.ptr, ds->wfrag.ptr, ds->wb2.ptr,
                                       ctx->gen_counter.ptr, ctx->stream};
  const std::vector<double> vk = {(double)ds->serial, (double)n_par, (double)n_pop,
                                  (double)(seed & 0xFFFFFFFFull), (double)(seed >> 32),
                                  lambda_host[0], lambda_host[1], lambda_host[2], lambda_host[3],
                                  lambda_host[4], eta_m, eta_s, (double)ds->pop_variant};
  if (!G.exec || G.ptr_key != pk || G.val_key != vk) {
    // the previous graph may still be running on the stream
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return check_hip(ctx, e, "waiting for the stream");
    G.release();
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return check_hip(ctx, e, "creating the capture stream");
    hipStream_t user = ctx->stream;
    const bool timing = ctx->timer.on;
    ctx->stream = cap;
    ctx->timer.on = false;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const int nb = (n_par + 3) / 4;
      launch_kernel(ctx, false, false, k_snes_sample, dim3(blocks_for(nb, kBlock), n_pop),
                    dim3(kBlock), n_par, (const float*)m_dev, (const float*)s_dev,
                    (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32), 0u,
                    (const int*)ctx->gen_counter.ptr, r_dev, Z_dev);
      hipError_t le = enqueue_population_loss(ctx, ds, n_pop, Z_dev, lambda_host, loss_dev,
                                              ds->pop_variant);
      launch_kernel(ctx, false, false, k_snes_update, dim3(blocks_for(n_par, kBlock)),
                    dim3(kBlock), n_par, n_pop, m_dev, s_dev, (const float*)r_dev,
                    (const double*)loss_dev, eta_m, eta_s);
      launch_kernel(ctx, false, false, k_snes_record, dim3(1), dim3(64), n_pop,
                    (const double*)loss_dev, ctx->gen_counter.ptr, best_dev);
      if (le == hipSuccess) le = hipGetLastError();
      hipGraph_t graph = nullptr;
      e = hipStreamEndCapture(cap, &graph);
      if (e == hipSuccess && le != hipSuccess) e = le;
      if (e == hipSuccess) {
        G.graph = graph;
        e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
      } else if (graph) {
        (void)hipGraphDestroy(graph);
      }
    }
    ctx->stream = user;
    ctx->timer.on = timing;
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
      G.release();
      return check_hip(ctx, e, "capturing the SNES generation");
    }
    G.ptr_key = pk;
    G.val_key = vk;
  }
  launch_kernel(ctx, false, false, k_set_counter, dim3(1), dim3(64), ctx->gen_counter.ptr,
                generation);
  e = hipGetLastError();
  for (int g = 0; g < n_gen && e == hipSuccess; ++g) e = hipGraphLaunch(G.exec, ctx->stream);
  return check_hip(ctx, e, "launching SNES generations");
}

}  // extern "C"
