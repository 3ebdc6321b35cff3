// Population evaluation over a training set (Sec. II E) on gfx950.
//
// Training positions do not change between generations, so everything that
// depends on geometry alone is computed once per dataset:
//   * the pairs inside a cutoff, compacted per atom (those inside r_c^A of
//     the angular list part first, then the rest inside r_c^R), each as a
//     record (float32 displacement r_ij, index of its reverse record);
//   * every atom's descriptor q_i and angular moments c_nlm (factorised form
//     of Eq. qinl), 149 floats.
// A generation then needs, per (atom, individual), only the network (Eqs.
// nn1, nn2), the coefficients a_nlm = 2 dU/dq_nl c_nlm and the partial forces
// (Sec. II D), followed by one block per (structure, individual) that forms
// F_i = sum_j p_ij - sum_j p_ji, the structure's energy and virial (Sec.
// II A) and the squared errors of the loss (Sec. II E), summed in float64 in
// a fixed order.
#include "nep_terms.h"

namespace nep {
namespace {

constexpr int NR = 9, NA = 5, LMAX = 4, NNEU = 30;
using M = Model<NR, NA, LMAX>;
constexpr int NDES = M::kNDES;             // 29
constexpr int NLM = M::kNLM;               // 24
constexpr int kDesc = NDES + NA * NLM;     // 149 cached floats per atom
constexpr int kDescRow = 152;              // padded row (float4 reads)

inline unsigned blocks_for(size_t work, int block) { return (unsigned)((work + block - 1) / block); }

// Pair classification in float32 (the same in both directions of a pair):
// 2 = inside r_c^A and in the angular part of the list, 1 = inside r_c^R
// only, 0 = outside.  cidx[s][i] = compacted index of slot s or -1.
__global__ void k_pair_classes(int N, const double* __restrict__ pos, const double* __restrict__ boxes,
                               const int* __restrict__ struct_of, const uint32_t* __restrict__ nl,
                               const int* __restrict__ cnt_r, const int* __restrict__ cnt_a,
                               float rca2, float rcr2, int* __restrict__ cidx,
                               int* __restrict__ n_ang, int* __restrict__ n_in) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double* H = boxes + 9 * (size_t)struct_of[i];
  const double xi = pos[i], yi = pos[N + i], zi = pos[2 * N + i];
  const int cr = cnt_r[i], ca = cnt_a[i];
  int k = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int s = 0; s < cr; ++s) {
      const size_t idx = (size_t)s * N + i;
      int j;
      float dx, dy, dz;
      displacement(nl[idx], pos, N, xi, yi, zi, H, j, dx, dy, dz);
      const float r2 = pair_r2(dx, dy, dz);
      const int cls = (s < ca && r2 < rca2) ? 2 : (r2 < rcr2 ? 1 : 0);
      if (pass == 0) {
        cidx[idx] = cls == 2 ? k++ : -1;
      } else if (cls == 1) {
        cidx[idx] = k++;
      }
    }
    if (pass == 0) n_ang[i] = k;
  }
  n_in[i] = k;
}

// rec[c][i] = (r_ij as float32, index of the reverse record c' N + j) for
// every compacted pair c of atom i.
__global__ void k_pair_records(int N, int cap, const double* __restrict__ pos,
                               const double* __restrict__ boxes, const int* __restrict__ struct_of,
                               const uint32_t* __restrict__ nl, const int* __restrict__ cnt_r,
                               const int* __restrict__ rev, const int* __restrict__ cidx,
                               float4* __restrict__ rec, int* __restrict__ flags) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)N * cap) return;
  const int i = (int)(idx % (size_t)N);
  const int s = (int)(idx / (size_t)N);
  if (s >= cnt_r[i]) return;
  const int c = cidx[idx];
  if (c < 0) return;
  const double* H = boxes + 9 * (size_t)struct_of[i];
  int j;
  float dx, dy, dz;
  displacement(nl[idx], pos, N, pos[i], pos[N + i], pos[2 * N + i], H, j, dx, dy, dz);
  int cr = cidx[(size_t)rev[idx] * N + j];
  int dst = cr * N + j;
  if (cr < 0) {  // lists cut at their capacity: keep the write inside this record
    flags[kFlagReverse] = 1;
    dst = c * N + i;
  }
  rec[(size_t)c * N + i] = make_float4(dx, dy, dz, __int_as_float(dst));
}

// desc[i][0..29) = q_i, desc[i][29 + n 24 + m] = c_nlm (L lanes per atom).
template <int L>
__global__ __launch_bounds__(kBlock) void k_ds_descriptors(int N, const float4* __restrict__ rec,
                                                           const int* __restrict__ n_ang,
                                                           const int* __restrict__ n_in,
                                                           float rc_r, float rc_a,
                                                           float* __restrict__ desc) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gid / L;
  const int lane = gid % L;
  const bool active = i < N;
  const int na = active ? n_ang[i] : 0, ni = active ? n_in[i] : 0;
  const float rcr_inv = 1.f / rc_r, rca_inv = 1.f / rc_a;
  float q[NDES];
  float c[NA][NLM];
#pragma unroll
  for (int v = 0; v < NDES; ++v) q[v] = 0.f;
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int m = 0; m < NLM; ++m) c[a][m] = 0.f;
  for (int k = lane; k < ni; k += L) {
    const float4 p = rec[(size_t)k * N + i];
    pair_descriptor<NR, NA, LMAX>(p.x, p.y, p.z, true, k < na, rcr_inv, rca_inv, q, c);
  }
#pragma unroll
  for (int a = 0; a < NR; ++a) q[a] = group_sum<L>(q[a]);
  radial_finish<NR>(q);
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int m = 0; m < NLM; ++m) c[a][m] = group_sum<L>(c[a][m]);
  angular_invariants<NR, NA, LMAX>(c, q);
  if (!active || lane != 0) return;
  float d[kDescRow];
#pragma unroll
  for (int v = 0; v < NDES; ++v) d[v] = q[v];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int m = 0; m < NLM; ++m) d[NDES + a * NLM + m] = c[a][m];
#pragma unroll
  for (int v = kDesc; v < kDescRow; ++v) d[v] = 0.f;
  float4* d4 = reinterpret_cast<float4*>(desc + (size_t)i * kDescRow);
#pragma unroll
  for (int t = 0; t < kDescRow / 4; ++t)
    d4[t] = make_float4(d[4 * t], d[4 * t + 1], d[4 * t + 2], d[4 * t + 3]);
}

// Pass 1 of every individual k = blockIdx.x on the atoms of block y: network,
// coefficients and partial forces, written to the reverse records of
// pin + k pstride; fown = sum_j p_ij and U per atom.
template <int L>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_pop_partials(
    int N, const float4* __restrict__ rec, const int* __restrict__ n_ang,
    const int* __restrict__ n_in, const float* __restrict__ desc, const float* __restrict__ Z,
    int n_par, float rc_r, float rc_a, Partial3* __restrict__ pin, size_t pstride,
    float* __restrict__ fown, float* __restrict__ U) {
  __shared__ float4 rows[NetRows<NDES, NNEU>::kFloat4];
  __shared__ float b2;
  // logical (individual, atom block), contiguous atom blocks per XCD
  const unsigned lb = xcd_block(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
  const size_t k = lb % gridDim.x;
  const unsigned by = lb / gridDim.x;
  load_net_rows<NDES, NNEU>(Z + k * (size_t)n_par, rows, &b2);
  pin += k * pstride;
  fown += k * 3 * (size_t)N;
  U += k * (size_t)N;
  __syncthreads();
  const int gid = (int)by * blockDim.x + threadIdx.x;
  const int i = gid / L;
  const int lane = gid % L;
  const bool active = i < N;
  const int ii = active ? i : 0;
  const int na = active ? n_ang[i] : 0, ni = active ? n_in[i] : 0;
  const float rcr_inv = 1.f / rc_r, rca_inv = 1.f / rc_a;
  float q[NDES];
  float c[NA][NLM];
  {
    const float4* d4 = reinterpret_cast<const float4*>(desc + (size_t)ii * kDescRow);
    float d[kDescRow];
#pragma unroll
    for (int t = 0; t < kDescRow / 4; ++t) {
      const float4 v = d4[t];
      d[4 * t] = v.x;
      d[4 * t + 1] = v.y;
      d[4 * t + 2] = v.z;
      d[4 * t + 3] = v.w;
    }
#pragma unroll
    for (int v = 0; v < NDES; ++v) q[v] = d[v];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int m = 0; m < NLM; ++m) c[a][m] = d[NDES + a * NLM + m];
  }
  float dq[NDES];
  float u;
  network<NDES, NNEU, L>(q, rows, b2, lane, dq, u);
  if (active && lane == 0) U[i] = u;
  angular_coefficients<NR, NA, LMAX>(dq, c);
  const float dqs = radial_dq_sum<NR>(dq);
  float fx = 0.f, fy = 0.f, fz = 0.f;
  for (int t = lane; t < ni; t += L) {
    const float4 p = rec[(size_t)t * N + i];
    float px, py, pz;
    pair_force<NR, NA, LMAX>(p.x, p.y, p.z, true, t < na, rcr_inv, rca_inv, dq, dqs, c, px, py,
                             pz);
    fx += px;
    fy += py;
    fz += pz;
    pin[(size_t)(unsigned)__float_as_int(p.w)] = Partial3{px, py, pz};
  }
  fx = group_sum<L>(fx);
  fy = group_sum<L>(fy);
  fz = group_sum<L>(fz);
  if (active && lane == 0) {
    fown[i] = fx;
    fown[N + i] = fy;
    fown[2 * N + i] = fz;
  }
}

// Pass 2 and the loss sums of individual k = blockIdx.x on structure
// s = blockIdx.y: per atom F_i = sum_j p_ij - sum_j p_ji and
// W_i = sum_j r_ij (x) p_ji; per structure
// sq[(k S + s) 3 + (0, 1, 2)] = (((U_s - E_s)/N_s)^2, sum_i |F_i - F_i^tar|^2,
// sum over xx yy zz xy yz zx of ((W_s - W_s^tar)/N_s)^2, or 0 without a target).
template <int L>
__global__ __launch_bounds__(kBlock) void k_pop_struct(
    int N, int S, const int* __restrict__ off, const float4* __restrict__ rec,
    const int* __restrict__ n_in, const Partial3* __restrict__ pin, size_t pstride,
    const float* __restrict__ fown, const float* __restrict__ U, const double* __restrict__ f_tar,
    const double* __restrict__ e_tar, const double* __restrict__ w_tar,
    const int* __restrict__ has_v, double* __restrict__ sq) {
  __shared__ double sw[kBlock / 64][8];
  __shared__ double tot[8];
  // logical (individual, structure), contiguous structures per XCD
  const unsigned lb = xcd_block(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
  const size_t k = lb % gridDim.x;
  const int s = (int)(lb / gridDim.x);
  pin += k * pstride;
  fown += k * 3 * (size_t)N;
  U += k * (size_t)N;
  const int a0 = off[s], a1 = off[s + 1];
  const int lane = threadIdx.x % L;
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  for (int base = a0; base < a1; base += kBlock / L) {
    const int i = base + (int)threadIdx.x / L;
    const bool active = i < a1;
    const int ni = active ? n_in[i] : 0;
    float f0 = 0.f, f1 = 0.f, f2 = 0.f;
    float w[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) w[q] = 0.f;
    for (int t = lane; t < ni; t += L) {
      const size_t idx = (size_t)t * N + i;
      const float4 r = rec[idx];
      const Partial3 p = pin[idx];
      f0 -= p.x;
      f1 -= p.y;
      f2 -= p.z;
      w[0] += r.x * p.x;
      w[1] += r.x * p.y;
      w[2] += r.x * p.z;
      w[3] += r.y * p.x;
      w[4] += r.y * p.y;
      w[5] += r.y * p.z;
      w[6] += r.z * p.x;
      w[7] += r.z * p.y;
      w[8] += r.z * p.z;
    }
    f0 = group_sum<L>(f0);
    f1 = group_sum<L>(f1);
    f2 = group_sum<L>(f2);
#pragma unroll
    for (int q = 0; q < 9; ++q) w[q] = group_sum<L>(w[q]);
    if (active && lane == 0) {
      const double F0 = (double)(f0 + fown[i]) - f_tar[i];
      const double F1 = (double)(f1 + fown[N + i]) - f_tar[N + i];
      const double F2 = (double)(f2 + fown[2 * N + i]) - f_tar[2 * N + i];
      acc[0] += (double)U[i];
      acc[1] += F0 * F0 + F1 * F1 + F2 * F2;
      acc[2] += (double)w[0];  // xx
      acc[3] += (double)w[4];  // yy
      acc[4] += (double)w[8];  // zz
      acc[5] += (double)w[1];  // xy
      acc[6] += (double)w[5];  // yz
      acc[7] += (double)w[6];  // zx
    }
  }
  const double v = block_sum<8>(acc, sw);
  if (threadIdx.x < 8) tot[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double ns = (double)(a1 - a0);
    const double de = (tot[0] - e_tar[s]) / ns;
    double dv = 0.0;
    if (has_v[s])
      for (int c = 0; c < 6; ++c) {
        const double d = (tot[2 + c] - w_tar[6 * s + c]) / ns;
        dv += d * d;
      }
    double* o = sq + (k * S + s) * 3;
    o[0] = de * de;
    o[1] = tot[1];
    o[2] = dv;
  }
}

template <int L>
void launch_pop(nep_ctx ctx, nep_dataset ds, int n_pop, const float* Z, bool first) {
  const int N = ds->N, S = ds->S;
  const unsigned nb = blocks_for((size_t)N * L, kBlock);
  const size_t pstride = (size_t)ds->cap * N;
  launch_kernel(ctx, first, false, k_pop_partials<L>, dim3(n_pop, nb), dim3(kBlock), N,
                (const float4*)ds->prec.ptr, (const int*)ds->pn_ang.ptr, (const int*)ds->pn_in.ptr,
                (const float*)ds->desc.ptr, Z, ctx->n_par, (float)ds->rc_r, (float)ds->rc_a,
                ds->pin.ptr, pstride, ds->fown.ptr, ds->U.ptr);
  // 2 lanes per atom: 3.33 ms per generation on the 1000-structure set
  // against 3.41 (4 lanes), 3.55 (8) and 3.81 (16); 1 lane ties with 2
  launch_kernel(ctx, false, false, k_pop_struct<2>, dim3(n_pop, S), dim3(kBlock), N, S,
                (const int*)ds->off.ptr, (const float4*)ds->prec.ptr, (const int*)ds->pn_in.ptr,
                (const Partial3*)ds->pin.ptr, pstride, (const float*)ds->fown.ptr,
                (const float*)ds->U.ptr, (const double*)ds->f_tar.ptr,
                (const double*)ds->e_tar.ptr, (const double*)ds->w_tar.ptr,
                (const int*)ds->has_v.ptr, ds->struct_sq.ptr);
}

}  // namespace

hipError_t prepare_dataset_geometry(nep_ctx ctx, nep_dataset ds) {
  const int N = ds->N, cap = ds->cap;
  const size_t ncap = (size_t)N * cap;
  hipError_t e = ds->prec.ensure(ncap);
  if (e == hipSuccess) e = ds->pcidx.ensure(ncap);
  if (e == hipSuccess) e = ds->pn_ang.ensure(N);
  if (e == hipSuccess) e = ds->pn_in.ensure(N);
  if (e == hipSuccess) e = ds->desc.ensure((size_t)kDescRow * N);
  if (e != hipSuccess) return e;
  const float rca = (float)ds->rc_a, rcr = (float)ds->rc_r;
  hipStream_t st = ctx->stream;
  k_pair_classes<<<blocks_for(N, 64), 64, 0, st>>>(
      N, ds->pos.ptr, ds->boxes.ptr, ds->struct_of.ptr, ds->nl.ptr, ds->cnt_r.ptr, ds->cnt_a.ptr,
      rca * rca, rcr * rcr, ds->pcidx.ptr, ds->pn_ang.ptr, ds->pn_in.ptr);
  k_pair_records<<<blocks_for(ncap, kBlock), kBlock, 0, st>>>(
      N, cap, ds->pos.ptr, ds->boxes.ptr, ds->struct_of.ptr, ds->nl.ptr, ds->cnt_r.ptr,
      ds->rev.ptr, ds->pcidx.ptr, ds->prec.ptr, ctx->flags.ptr);
  k_ds_descriptors<4><<<blocks_for((size_t)N * 4, kBlock), kBlock, 0, st>>>(
      N, ds->prec.ptr, ds->pn_ang.ptr, ds->pn_in.ptr, rcr, rca, ds->desc.ptr);
  return hipGetLastError();
}

int population_variants() { return 3; }
int population_lanes(int variant) { return variant == 0 ? 2 : (variant == 1 ? 4 : 8); }

hipError_t launch_population(nep_ctx ctx, nep_dataset ds, int n_pop, const float* Z, int variant,
                             bool first) {
  if (ds->N == 0 || n_pop == 0) return hipSuccess;
  if (blocks_for((size_t)ds->N * 8, kBlock) > 65535 || ds->S > 65535 || n_pop > 65535)
    return hipErrorInvalidConfiguration;
  switch (variant) {
    case 0:
      launch_pop<2>(ctx, ds, n_pop, Z, first);
      break;
    case 2:
      launch_pop<8>(ctx, ds, n_pop, Z, first);
      break;
    default:
      launch_pop<4>(ctx, ds, n_pop, Z, first);
  }
  return hipGetLastError();
}

}  // namespace nep
