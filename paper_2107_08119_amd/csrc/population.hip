// Population evaluation over a training set (Sec. II E) on gfx950: the loss
// of every parameter vector of a population over every structure, in two
// launches per population, with the dense contractions on the matrix cores.
//
// Training positions do not change between generations, so everything that
// depends on geometry alone is computed once per dataset:
//   * the pairs inside a cutoff, compacted per atom (those inside r_c^A of
//     the angular list part first, then the rest inside r_c^R), each as a
//     record (float32 displacement r_ij, index of its reverse record);
//   * every atom's descriptor q_i and angular moments c_nlm (factorised form
//     of Eq. qinl);
//   * per pair, the derivative of atom i's descriptor with respect to r_ij,
//     D_ij[b][nu] = dq^i_nu / d(r_ij)_b (Sec. II D).  It depends on geometry
//     only (the angular part through c_nlm), so the partial force of any
//     parameter vector is the contraction p_ij = sum_nu D_ij[.][nu] dU/dq_nu.
//     Its radial part is g_n'(r) r_ij/r, stored as the scalars g_n'; the
//     angular part is 3 x 20 numbers per angular pair;
//   * per atom, G_i = sum_j D_ij (3 x 29: sum_j p_ij = G_i dU/dq) and
//     V_i[a][b] = -sum_j (r_ij)_a D_ij[b] (9 x 29: the structure's virial is
//     sum_i V_i dU/dq, since summing W_i = sum_j r_ij (x) p_ji over a
//     structure visits every pair in both directions, r_ji = -r_ij).
// These operands are stored in the fragment order of the 16x16x4 float32
// matrix instruction, so one wave-wide load fetches one step's operand.
//
// A generation then runs:
//   * the network kernel: per individual k, act^T = W1_k Q^T (rows neurons,
//     columns atoms), tanh, U_i, and dU/dq = (w2 sech^2(act)) W1_k as two
//     products on the matrix cores (Eqs. nn1, nn2 and their input gradient);
//   * the contraction kernel: one block per tile of whole structures keeps
//     the forces of every atom of the tile for every individual in LDS.  Wave
//     w owns the individuals k = w mod 4, sixteen per matrix tile, and for
//     each atom i multiplies D_i (rows: pair components) by dU/dq_i (columns:
//     individuals); each product element p_ij goes to F_j with an LDS add
//     (F_i = sum_j p_ij - sum_j p_ji, Sec. II A), G_i and V_i give the own
//     force and the virial.  No partial force goes to memory.  At the end of
//     each structure the wave forms its energy, force and virial errors in
//     float64 in a fixed order (Sec. II E).  Only wave w touches the forces
//     of its individuals, so the sums do not depend on scheduling.
#include <algorithm>
#include <vector>

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

// ------------------------------------------------- population operands

typedef float f32x4 __attribute__((ext_vector_type(4)));

// D[16x4] x B[4x16] + C on the matrix cores: lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and holds C[4 (l/16) + r][l%16] in element r.
__device__ __forceinline__ f32x4 mma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Padded descriptor order of the population kernels: radial components at
// 0..8, zeros at 9..11, angular components nu = 9..28 at nu + 3 = 12..31, so
// that a lane's K steps of the angular product (K index 12 + 4 s + l/16) are
// a subset of those of the full product (4 s + l/16).
constexpr int kQ = 32;
constexpr int kAng0 = 12;
__host__ __device__ constexpr int padded(int v) { return v < NR ? v : v + (kAng0 - NR); }

// Fragment chunks (64 floats) per atom: the own-force/virial tile (8 K steps
// over the padded descriptor), ns radial tiles of 16 pairs (3 K steps: the
// nine g_n' and three zeros), and per block of 16 angular pairs three
// angular tiles, one per component x, y, z (5 K steps over the angular
// part).  Row r of radial tile b and of the angular tiles of block b belong
// to the same pair 16 b + r, so a lane holds both parts of a pair's partial
// force and adds them before they go to LDS.
constexpr int kGSteps = 8, kSSteps = 3, kASteps = 5;
__host__ __device__ inline int radial_tiles(int pairs) { return (pairs + 15) / 16; }
__host__ __device__ inline int angular_tiles(int ang) { return 3 * ((ang + 15) / 16); }
__host__ __device__ inline int atom_chunks(int pairs, int ang) {
  return kGSteps + kSSteps * radial_tiles(pairs) + kASteps * angular_tiles(ang);
}

// Fixed-point accumulators of a tile in LDS (162,816 bytes): forces
// [atom][3][KC] and structure virials [structure][9][KC], 32-bit integers.
constexpr int kLdsInts = 40704;
constexpr int kTileTarget = 64;

// Memory order of dU/dq within an (atom, individual) row of 32: padded
// index kappa is stored at dq_slot(kappa) = 8 (kappa % 4) + kappa / 4, so the
// 8 values a contraction lane multiplies (kappa = 4 q + h, q = 0..7) are
// contiguous, and the network kernel's lane writes the pair kappa, kappa + 4
// (its two output tiles) as one 8-byte store.
__host__ __device__ constexpr int dq_slot(int kappa) { return 8 * (kappa % 4) + kappa / 4; }
// the padded index of output column col of the network's second product, tile nt
__host__ __device__ constexpr int dq_kappa(int col, int nt) {
  return 8 * (col / 4) + col % 4 + 4 * nt;
}

__global__ void k_pop_qpad(int N, const float* __restrict__ desc, float* __restrict__ qpad) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)N * kQ) return;
  const int i = (int)(t / kQ), v = (int)(t % kQ);
  float q = 0.f;
  if (v < NR)
    q = desc[(size_t)i * kDescRow + v];
  else if (v >= kAng0)
    q = desc[(size_t)i * kDescRow + v - (kAng0 - NR)];
  qpad[t] = q;
}

// One thread per (atom i, descriptor component nu < 29): D_ij[.][nu] for
// every pair of i, written into i's radial or angular fragment chunks, and
// row nu of G_i and V_i.  The thread of nu = 0 also writes the pair records
// (r_ij/r_ij, offset 3 kcs j of the receiver's force accumulators in the
// tile).  pfrag must be zero before.
__global__ __launch_bounds__(kBlock) void k_pop_geo(
    int N, int kcs, const float4* __restrict__ rec, const int4* __restrict__ pmeta,
    const float* __restrict__ desc, const int* __restrict__ struct_of,
    const int* __restrict__ stile0, float rc_r, float rc_a, float* __restrict__ pfrag,
    float4* __restrict__ ppair) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gid / 32, v = gid % 32;
  if (i >= N || v >= NDES) return;
  const int4 m = pmeta[i];
  const size_t dbase = (size_t)(unsigned)m.x;
  const int P = m.z, A = m.w;
  const int ns = radial_tiles(P);
  const int t0 = stile0[struct_of[i]];
  float G[3] = {0.f, 0.f, 0.f};
  float V[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) V[q] = 0.f;
  if (v < NR) {
    const float rcr_inv = 1.f / rc_r;
    for (int p = 0; p < P; ++p) {
      const float4 e = rec[(size_t)p * N + i];
      const float r2 = pair_r2(e.x, e.y, e.z);
      const float rinv = __builtin_amdgcn_rsqf(r2);
      const float r = r2 * rinv;
      float fc, dfc, dxdr, T[NR], dT[NR];
      chebyshev_terms<NR>(r, rcr_inv, fc, dfc, dxdr, T, dT);
      const float gp = 0.5f * (dfc * (T[v] + 1.f) + fc * dxdr * dT[v]);
      const size_t chunk = dbase + kGSteps + (size_t)kSSteps * (p / 16) + v / 4;
      pfrag[chunk * 64 + (v % 4) * 16 + p % 16] = gp;
      const float d[3] = {gp * e.x * rinv, gp * e.y * rinv, gp * e.z * rinv};
      const float rv[3] = {e.x, e.y, e.z};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        G[b] += d[b];
#pragma unroll
        for (int a = 0; a < 3; ++a) V[3 * a + b] -= rv[a] * d[b];
      }
      if (v == 0) {
        const int j = (int)((unsigned)__float_as_int(e.w) % (unsigned)N);
        ppair[(size_t)m.y + p] =
            make_float4(e.x * rinv, e.y * rinv, e.z * rinv, __int_as_float((j - t0) * 3 * kcs));
      }
    }
  } else {
    const int n = (v - NR) / LMAX, l = (v - NR) % LMAX + 1;
    const float rca_inv = 1.f / rc_a;
    const float* c = desc + (size_t)i * kDescRow + NDES + n * NLM;
    for (int a = 0; a < A; ++a) {
      const float4 e = rec[(size_t)a * N + i];
      const float r2 = pair_r2(e.x, e.y, e.z);
      const float rinv = __builtin_amdgcn_rsqf(r2);
      const float r = r2 * rinv;
      float g[NA], dg[NA];
      radial_basis<NA, true>(r, rca_inv, g, dg);
      const float x = e.x * rinv, y = e.y * rinv, z = e.z * rinv;
      const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
      const float xyz = xy * z;
      (void)xyz;
      // s_y = sum_m c_nlm Yhat_lm, s_g = sum_m c_nlm grad Yhat_lm (l fixed)
      float sy = 0.f, sgx = 0.f, sgy = 0.f, sgz = 0.f;
#define NEP_DG(idx, YV, GX, GY, GZ)                      \
  if ((idx) >= l * l - 1 && (idx) < (l + 1) * (l + 1) - 1) { \
    const float cm = c[idx];                              \
    sy += cm * (YV);                                      \
    sgx += cm * (GX);                                     \
    sgy += cm * (GY);                                     \
    sgz += cm * (GZ);                                     \
  }
      NEP_YLM_TABLE(NEP_DG)
#undef NEP_DG
      // d/dr_ij [g_n(r) Yhat(r/|r|)] = g_n' Yhat u + g_n (grad Yhat - u (u.grad Yhat)) / r
      const float ug = x * sgx + y * sgy + z * sgz;
      const float d[3] = {2.f * (dg[n] * sy * x + g[n] * (sgx - x * ug) * rinv),
                          2.f * (dg[n] * sy * y + g[n] * (sgy - y * ug) * rinv),
                          2.f * (dg[n] * sy * z + g[n] * (sgz - z * ug) * rinv)};
      const float rv[3] = {e.x, e.y, e.z};
      const int kap = v - NR;  // K index within the angular product
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const size_t chunk = dbase + kGSteps + (size_t)kSSteps * ns +
                             (size_t)kASteps * (3 * (a / 16) + b) + kap / 4;
        pfrag[chunk * 64 + (kap % 4) * 16 + a % 16] = d[b];
        G[b] += d[b];
#pragma unroll
        for (int q = 0; q < 3; ++q) V[3 * q + b] -= rv[q] * d[b];
      }
    }
  }
  // own-force / virial tile: rows 0..2 = G, rows 3..11 = V (row-major ab)
  const int kap = padded(v);
  float* gt = pfrag + (dbase + kap / 4) * 64 + (kap % 4) * 16;
#pragma unroll
  for (int b = 0; b < 3; ++b) gt[b] = G[b];
#pragma unroll
  for (int q = 0; q < 9; ++q) gt[3 + q] = V[q];
}

// The largest of a and b, NaN if either is NaN (so a non-finite dU/dq reaches
// the bound and marks the individual).
__device__ __forceinline__ float max_nan(float a, float b) { return (b > a || b != b) ? b : a; }

// The network weights of individual k = blockIdx.x in the lane order of the
// network kernel's two products: wf[(k 12 + q) 64 + lane] (float4) holds for
// lane (col, h) = (lane % 16, lane / 16)
//   q 0..3:  W1[16 mt + col][nu(4 s + h)], the first product's A (mt, s),
//   q 4..7:  W1[16 (s / 4) + 4 h + s % 4][nu(16 nt + col)], the second's B,
//   q 8..11: b1 and w2 of the lane's neurons 16 mt + 4 h + r,
// with nu(kappa) the descriptor component of padded index kappa and zeros for
// padding; wb2[k] = b2; dqbound[k] bounds |dU/dq| of individual k.
__global__ __launch_bounds__(64) void k_pop_wfrag(int n_par, const float* __restrict__ Z,
                                                  float4* __restrict__ wf,
                                                  float* __restrict__ wb2,
                                                  float* __restrict__ dqbound) {
  const int k = blockIdx.x, l = threadIdx.x, col = l & 15, h = l >> 4;
  const float* z = Z + (size_t)k * n_par;
  // |dU/dq_nu| = |sum_mu w2_mu sech^2(a_mu) W1[mu][nu]| <= sum_mu |w2_mu W1[mu][nu]|
  // (sech^2 <= 1): a bound for every atom; NaN or infinite with the weights
  float bnd = 0.f;
  if (l < NDES)
    for (int mu = 0; mu < NNEU; ++mu)
      bnd += fabsf(z[NNEU * (NDES + 1) + mu] * z[mu * NDES + l]);
  for (int d = 32; d > 0; d >>= 1) bnd = max_nan(bnd, __shfl_xor(bnd, d, 64));
  if (l == 0) dqbound[k] = bnd;
  auto w1 = [&](int mu, int kp) {
    const int nu = kp < NR ? kp : kp - (kAng0 - NR);
    return (mu < NNEU && (kp < NR || kp >= kAng0)) ? z[mu * NDES + nu] : 0.f;
  };
  float f[48];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int st = 0; st < 8; ++st) f[8 * mt + st] = w1(16 * mt + col, 4 * st + h);
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int st = 0; st < 8; ++st)
      f[16 + 8 * nt + st] = w1(16 * (st / 4) + 4 * h + (st % 4), dq_kappa(col, nt));
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mu = 16 * mt + 4 * h + r;
      f[32 + 4 * mt + r] = mu < NNEU ? z[NNEU * NDES + mu] : 0.f;
      f[40 + 4 * mt + r] = mu < NNEU ? z[NNEU * (NDES + 1) + mu] : 0.f;
    }
#pragma unroll
  for (int q = 0; q < 12; ++q)
    wf[((size_t)k * 12 + q) * 64 + l] = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
  if (l == 0) wb2[k] = z[NNEU * (NDES + 2)];
}

// dU/dq of every individual on atoms [16 CT w', 16 CT (w' + 1)) for wave w':
// act^T = W1_k Q^T (rows: neurons in two tiles of 16; columns: atoms), the
// neurons' tanh, U_i, and dU/dq_i = sum_mu w2_mu sech^2(act_mu) W1_k[mu] as
// a product whose K order (neurons) follows what each lane already holds,
// so G = w2 sech^2 never moves between lanes.  Each individual's weight
// fragments are loaded while the previous individual is multiplied.
// dq [N][n_pop][32] (padded order, zeros at 9..11), U [n_pop][N].
// Individuals per wave of the network kernel: the population is split into
// chunks over blockIdx.y, so that the grid has many more waves than the
// machine holds at once (whole waves of all individuals left the last round
// of waves mostly empty).
constexpr int kNetChunk = 10;

template <int CT>
__global__ __launch_bounds__(kBlock) void k_pop_net(int N, int n_pop,
                                                    const float* __restrict__ qpad,
                                                    const float4* __restrict__ wf,
                                                    const float* __restrict__ wb2,
                                                    float* __restrict__ dq,
                                                    float* __restrict__ U) {
  const int l = threadIdx.x & 63, col = l & 15, h = l >> 4;
  const int a0 = (blockIdx.x * (kBlock / 64) + threadIdx.x / 64) * 16 * CT;
  if (a0 >= N) return;  // whole waves leave together
  // Q^T fragments: B[kappa = 4 s + h][atom = col]
  float qb[CT][8];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int a = a0 + 16 * ct + col;
#pragma unroll
    for (int s = 0; s < 8; ++s) qb[ct][s] = a < N ? qpad[(size_t)a * kQ + 4 * s + h] : 0.f;
  }
  // the individuals k_begin .. k_end - 1 of this wave (blockIdx.y chunk)
  const int k_begin = blockIdx.y * kNetChunk;
  const int k_end = min(n_pop, k_begin + kNetChunk);
  float4 nxt[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) nxt[q] = wf[((size_t)k_begin * 12 + q) * 64 + l];
  for (int k = k_begin; k < k_end; ++k) {
    float f[48];
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      f[4 * q] = nxt[q].x;
      f[4 * q + 1] = nxt[q].y;
      f[4 * q + 2] = nxt[q].z;
      f[4 * q + 3] = nxt[q].w;
    }
    const float b2 = wb2[k];
    const int kn = k + 1 < k_end ? k + 1 : k;
#pragma unroll
    for (int q = 0; q < 12; ++q) nxt[q] = wf[((size_t)kn * 12 + q) * 64 + l];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      f32x4 act[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        act[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 8; ++s) act[mt] = mma(f[8 * mt + s], qb[ct][s], act[mt]);
      }
      float gm[2][4];
      float u = 0.f;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float x = act[mt][r] - f[32 + 4 * mt + r];
          const float w2 = f[40 + 4 * mt + r];
          // tanh and 1 - tanh^2 from e = exp(-2|x|) (no cancellation)
          const float ea = __expf(-2.f * fabsf(x));
          const float inv = __builtin_amdgcn_rcpf(1.f + ea);
          const float th = copysignf((1.f - ea) * inv, x);
          u += w2 * th;
          gm[mt][r] = w2 * (4.f * ea * inv * inv);
        }
      u += __shfl_xor(u, 16, 64);
      u += __shfl_xor(u, 32, 64);
      const int a = a0 + 16 * ct + col;
      if (h == 0 && a < N) U[(size_t)k * N + a] = u - b2;
      f32x4 o[2];
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        o[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 8; ++s) o[nt] = mma(gm[s / 4][s % 4], f[16 + 8 * nt + s], o[nt]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ar = a0 + 16 * ct + 4 * h + r;
        if (ar < N) {
          // kappa = dq_kappa(col, 0) and dq_kappa(col, 1) = that + 4: adjacent slots
          float* d = dq + ((size_t)ar * n_pop + k) * kQ + dq_slot(dq_kappa(col, 0));
          *reinterpret_cast<float2*>(d) = make_float2(o[0][r], o[1][r]);
        }
      }
    }
  }
}

// Per atom: the largest 1-norm (over the K index) of its force rows (own
// force rows of the first tile, radial and angular rows) and of its virial
// rows.  A force contribution of individual k is at most the first times
// max |dU/dq_i|; a virial contribution the second.
__global__ void k_pop_norms(int N, const int4* __restrict__ pmeta, const float* __restrict__ pfrag,
                            float2* __restrict__ pnorm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int4 m = pmeta[i];
  const float* f = pfrag + (size_t)(unsigned)m.x * 64;
  const int P = m.z, A = m.w, ns = radial_tiles(P), na = angular_tiles(A);
  float fmax = 0.f, vmax = 0.f;
#pragma unroll 1
  for (int row = 0; row < 12; ++row) {
    float s = 0.f;
    for (int q = 0; q < kGSteps; ++q)
      for (int hh = 0; hh < 4; ++hh) s += fabsf(f[64 * q + 16 * hh + row]);
    if (row < 3)
      fmax = fmaxf(fmax, s);
    else
      vmax = fmaxf(vmax, s);
  }
  const float* fs = f + 64 * kGSteps;
#pragma unroll 1
  for (int p = 0; p < P; ++p) {
    float s = 0.f;
    for (int q = 0; q < kSSteps; ++q)
      for (int hh = 0; hh < 4; ++hh) s += fabsf(fs[64 * (kSSteps * (p / 16) + q) + 16 * hh + p % 16]);
    fmax = fmaxf(fmax, s);
  }
  const float* fa = fs + 64 * kSSteps * ns;
#pragma unroll 1
  for (int row = 0; row < 3 * A; ++row) {
    const int a = row / 3, b = row % 3;
    float s = 0.f;
    for (int q = 0; q < kASteps; ++q)
      for (int hh = 0; hh < 4; ++hh)
        s += fabsf(fa[64 * (kASteps * (3 * (a / 16) + b) + q) + 16 * hh + a % 16]);
    fmax = fmaxf(fmax, s);
  }
  (void)na;
  pnorm[i] = make_float2(fmax, vmax);
}

// Fixed-point exponents of a tile for individual k: a force component of
// the tile receives at most deg_t contributions of at most
// max_i (largest force-row 1-norm of i) dqbound_k, a structure's virial
// component at most sum_i (largest virial-row 1-norm of i) dqbound_k; values
// are stored as round(x 2^e) in 32 bits with e chosen so that these bounds
// stay below 2^30.  A non-finite bound gives e = kBadScale.
constexpr int kBadScale = -1000;

// floor(x + 1/2) as a 32-bit integer in one instruction (round half up; the
// fixed-point values stay below 2^30 in magnitude)
__device__ __forceinline__ int round_to_int(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}
__device__ __forceinline__ int fixed_exponent(float bound) {
  if (!(bound <= 3.0e38f)) return kBadScale;  // NaN or infinite
  if (bound <= 0.f) return 30;
  int e;
  (void)frexpf(bound, &e);  // bound < 2^e
  const int s = 30 - e;
  return s < -100 ? -100 : (s > 100 ? 100 : s);
}

// Fragment operands of one owner atom in the contraction kernel, all
// requested before the atom's first product (the pair records are read just
// before the products of their block: holding them from the start would cost
// 32 registers, and with them a third wave per SIMD).  Atoms with at most
// kFastPairs pairs and kFastAng angular pairs (two radial tiles, one block of
// angular tiles) are fetched whole; others read their further tiles as they
// are used.
constexpr int kFastPairs = 32, kFastAng = 16;
constexpr int kFastS = 2;
constexpr int kCols = 4;  // column tiles of 16 individuals per wave
struct AtomOps {
  float b[kCols][8];   // dU/dq of the lane's individuals, K index 4 q + h
  float g[kGSteps];    // own-force / virial tile
  float s[kFastS][kSSteps];
  float a[3][kASteps];   // angular tiles x, y, z of the first pair block
};

__device__ __forceinline__ bool fast_atom(int4 m) { return m.z <= kFastPairs && m.w <= kFastAng; }

// Every load is issued unconditionally (the operand arrays carry kPadChunks
// chunks and kPadPairs pair records of padding, so a tile or pair past the
// atom's own reads a neighbour's data or padding) and masked at use: with no
// branch between the loads, each operand waits only for itself.
constexpr int kPadChunks = 64, kPadPairs = 64;
__device__ __forceinline__ void fetch_atom(AtomOps& o, int4 m, int i, int n_pop,
                                           const float* const (&dqk)[kCols],
                                           const float* pfrag, const float4* ppair, int l,
                                           int h) {
  const size_t row = (size_t)i * n_pop * kQ;
#pragma unroll
  for (int c = 0; c < kCols; ++c) {  // kappa = 4 q + h at slots 8 h + q
    const float4 lo = *reinterpret_cast<const float4*>(dqk[c] + row);
    const float4 hi = *reinterpret_cast<const float4*>(dqk[c] + row + 4);
    o.b[c][0] = lo.x;
    o.b[c][1] = lo.y;
    o.b[c][2] = lo.z;
    o.b[c][3] = lo.w;
    o.b[c][4] = hi.x;
    o.b[c][5] = hi.y;
    o.b[c][6] = hi.z;
    o.b[c][7] = hi.w;
  }
  const float* fr = pfrag + (size_t)(unsigned)m.x * 64 + l;
  const int ns = radial_tiles(m.z);
#pragma unroll
  for (int q = 0; q < kGSteps; ++q) o.g[q] = fr[64 * q];
#pragma unroll
  for (int tt = 0; tt < kFastS; ++tt)
#pragma unroll
    for (int q = 0; q < kSSteps; ++q) o.s[tt][q] = fr[64 * (kGSteps + kSSteps * tt + q)];
  const float* fa = fr + 64 * (kGSteps + kSSteps * ns);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int q = 0; q < kASteps; ++q) o.a[c][q] = fa[64 * (kASteps * c + q)];
}

// Forces, energies, virials and squared errors of individuals k0 .. k0+KC-1
// (KC <= 64) on the tile of structures tile_order[blockIdx.x].
// Phase 1: the waves take the tile's atoms in turn; for each atom and each
// column tile of 16 individuals they multiply the atom's operands by dU/dq
// and add every product element, as round(x 2^e) with the tile's exponent e
// of the individual, into 32-bit LDS accumulators of forces [atom][3][KC]
// and structure virials [structure][9][KC].  Integer sums do not depend on
// their order, so results are the same for any schedule.
// Phase 2: one unit per (structure, individual): lanes over the atoms form
// the energy, force and virial errors in float64 in a fixed order.
constexpr int kContractWaves = 12;
__global__ __launch_bounds__(64 * kContractWaves) void k_pop_contract(
    int N, int S, int k0, int KC, int kcs, int n_pop, const int* __restrict__ tile_order,
    const int* __restrict__ tile_off, const int* __restrict__ tile_s0,
    const int* __restrict__ off, const int* __restrict__ struct_of,
    const int4* __restrict__ pmeta, const float* __restrict__ pfrag,
    const float4* __restrict__ ppair, const float* __restrict__ dq, const float* __restrict__ U,
    const float2* __restrict__ tbound, const float* __restrict__ dqbound,
    const double* __restrict__ f_tar,
    const double* __restrict__ e_tar, const double* __restrict__ w_tar,
    const int* __restrict__ has_v, double* __restrict__ sq) {
  __shared__ int acc[kLdsInts];
  __shared__ int esc[2][64];
  const int t = tile_order[blockIdx.x];
  const int ta = tile_off[t], tb = tile_off[t + 1];
  const int s0 = tile_s0[t], s1 = tile_s0[t + 1];
  int* Fq = acc;                          // [atom][3][kcs]
  int* Wq = acc + (tb - ta) * 3 * kcs;    // [structure][9][kcs]
  const int n_acc = ((tb - ta) * 3 + (s1 - s0) * 9) * kcs;
  for (int x = threadIdx.x; x < n_acc; x += blockDim.x) acc[x] = 0;
  if (threadIdx.x < KC) {
    const float2 tb2 = tbound[t];
    const float bk = dqbound[k0 + threadIdx.x];
    esc[0][threadIdx.x] = fixed_exponent(tb2.x * bk);
    esc[1][threadIdx.x] = fixed_exponent(tb2.y * bk);
  }
  __syncthreads();
  const int w = threadIdx.x / 64, l = threadIdx.x & 63, col = l & 15, h = l >> 4;
  const float* dqk[kCols];
  float sF[kCols], rW[kCols];
  bool valid[kCols];
#pragma unroll
  for (int c = 0; c < kCols; ++c) {
    const int kl = 16 * c + col;
    valid[c] = kl < KC;
    const int k = k0 + (valid[c] ? kl : 0);
    dqk[c] = dq + (size_t)k * kQ + 8 * h;  // K index 4 q + h at slot 8 h + q
    const int eF = valid[c] ? esc[0][kl] : kBadScale, eW = valid[c] ? esc[1][kl] : kBadScale;
    // the force scale goes into dU/dq, so the products come out scaled; the
    // virial rows are rescaled by 2^(eW - eF).  A non-finite bound: every
    // contribution 0 (the loss is set to NaN below).
    const bool ok = eF != kBadScale && eW != kBadScale;
    sF[c] = ok ? ldexpf(1.f, eF) : 0.f;
    rW[c] = ok ? ldexpf(1.f, eW - eF) : 0.f;
  }
  auto add_q = [&](int* p, float x) { atomicAdd(p, round_to_int(x)); };

  // the pair block pb of atom i: radial tile v (rows: pairs) and, when the
  // block holds angular pairs, angular tiles ax, ay, az (same rows);
  // F_j -= u_ij v + (ax, ay, az) for the receiver j of each row.  Rows past
  // the atom's pairs have zero operands (their products are 0) and go to the
  // tile's first accumulator, so no lane branches.
  auto scatter_block = [&](const f32x4& v, const f32x4* va, bool ang, const float4 (&e)[4],
                           int pb, int P, int kl) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int dst = 16 * pb + 4 * h + r < P ? __float_as_int(e[r].w) : 0;
      int* fj = &Fq[dst + kl];
      float x = -e[r].x * v[r], y = -e[r].y * v[r], z = -e[r].z * v[r];
      if (ang) {
        x -= va[0][r];
        y -= va[1][r];
        z -= va[2][r];
      }
      add_q(fj, x);
      add_q(fj + kcs, y);
      add_q(fj + 2 * kcs, z);
    }
  };

  auto process = [&](AtomOps& o, int4 m, int i, int sl) {
    const int il = i - ta;
    const int P = m.z, A = m.w;
    const int ns = radial_tiles(P), nab = (A + 15) / 16;
#pragma unroll
    for (int c = 0; c < kCols; ++c)
#pragma unroll
      for (int q = 0; q < 8; ++q) o.b[c][q] *= sF[c];
    // the lane's rows 4 h + r of the own-force / virial tile: rows 0..2 the
    // own force, 3..11 the virial (row-major ab), 12..15 zero
    int gdst[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * h + r;
      gdst[r] = row < 3 ? (il * 3 + row) * kcs
                        : (row < 12 ? (int)(Wq - Fq) + (sl * 9 + row - 3) * kcs : il * 3 * kcs);
    }
#pragma unroll
    for (int c = 0; c < kCols; ++c) {
      f32x4 g = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < kGSteps; ++q) g = mma(o.g[q], o.b[c][q], g);
      if (!valid[c]) continue;
      const int kl = 16 * c + col;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        add_q(&Fq[gdst[r] + kl], 4 * h + r < 3 ? g[r] : g[r] * rW[c]);
    }
    if (fast_atom(m)) {
#pragma unroll
      for (int pb = 0; pb < kFastS; ++pb) {
        if (pb >= ns) break;
        const bool ang = pb < nab;
        float4 e[4];  // the rows' pair records, read while the products run
#pragma unroll
        for (int r = 0; r < 4; ++r) e[r] = ppair[(size_t)m.y + 16 * pb + 4 * h + r];
#pragma unroll
        for (int c = 0; c < kCols; ++c) {
          f32x4 v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < kSSteps; ++q) v = mma(o.s[pb][q], o.b[c][q], v);
          f32x4 va[3];
          if (ang) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              va[d] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
              for (int q = 0; q < kASteps; ++q) va[d] = mma(o.a[d][q], o.b[c][3 + q], va[d]);
            }
          }
          if (valid[c]) scatter_block(v, va, ang, e, pb, P, 16 * c + col);
        }
      }
      return;
    }
    // atoms with more pairs: the further operands read as they are used
    const float* fs = pfrag + (size_t)(unsigned)m.x * 64 + l + 64 * kGSteps;
    const float* fa = fs + 64 * kSSteps * ns;
    for (int pb = 0; pb < ns; ++pb) {
      float d[kSSteps], da[3][kASteps];
#pragma unroll
      for (int q = 0; q < kSSteps; ++q) d[q] = fs[64 * (kSSteps * pb + q)];
      const bool ang = pb < nab;
#pragma unroll
      for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int q = 0; q < kASteps; ++q)
          da[x][q] = ang ? fa[64 * (kASteps * (3 * pb + x) + q)] : 0.f;
      float4 e[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = 16 * pb + 4 * h + r;
        e[r] = ppair[(size_t)m.y + (p < P ? p : 0)];
      }
#pragma unroll
      for (int c = 0; c < kCols; ++c) {
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < kSSteps; ++q) v = mma(d[q], o.b[c][q], v);
        f32x4 va[3];
        if (ang) {
#pragma unroll
          for (int x = 0; x < 3; ++x) {
            va[x] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < kASteps; ++q) va[x] = mma(da[x][q], o.b[c][3 + q], va[x]);
          }
        }
        if (valid[c]) scatter_block(v, va, ang, e, pb, P, 16 * c + col);
      }
    }
  };

  // Phase 1: atoms ta + w, ta + w + kContractWaves, ...; all fragment
  // operands of an atom are requested before its first product (the other
  // waves on the SIMD cover the wait), its pair records just before the
  // products that use them
  // (the atom records are read with vector loads, threadIdx.y being 0: a
  // scalar load would have to wait for every LDS addition in flight)
  for (int i = ta + w; i < tb; i += kContractWaves) {
    int4 m = pmeta[i + threadIdx.y];
    m.x = __builtin_amdgcn_readfirstlane(m.x);
    m.y = __builtin_amdgcn_readfirstlane(m.y);
    m.z = __builtin_amdgcn_readfirstlane(m.z);
    m.w = __builtin_amdgcn_readfirstlane(m.w);
    const int sl = __builtin_amdgcn_readfirstlane(struct_of[i + threadIdx.y] - s0);
    AtomOps o;
    fetch_atom(o, m, i, n_pop, dqk, pfrag, ppair, l, h);
    process(o, m, i, sl);
  }
  __syncthreads();
  // Phase 2: unit (structure s, individual kl), lanes over atoms
  const int n_units = (s1 - s0) * KC;
  for (int u = w; u < n_units; u += kContractWaves) {
    const int s = s0 + u / KC, kl = u % KC, k = k0 + kl;
    const int i0 = off[s], i1 = off[s + 1];
    const int eF = esc[0][kl], eW = esc[1][kl];
    const double iF = eF == kBadScale ? 0.0 : ldexp(1.0, -eF);
    const double iW = eW == kBadScale ? 0.0 : ldexp(1.0, -eW);
    double eu = 0.0, ef = 0.0;
    for (int i = i0 + l; i < i1; i += 64) {
      eu += (double)U[(size_t)k * N + i];
      const int il = i - ta;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double d = (double)Fq[(il * 3 + c) * kcs + kl] * iF - f_tar[(size_t)c * N + i];
        ef += d * d;
      }
    }
    for (int d = 32; d > 0; d >>= 1) {
      eu += __shfl_xor(eu, d, 64);
      ef += __shfl_xor(ef, d, 64);
    }
    if (l == 0) {
      const double ns_inv = 1.0 / (double)(i1 - i0);
      double ev = 0.0;
      if (has_v[s]) {
        // targets xx yy zz xy yz zx = row-major components 0, 4, 8, 1, 5, 6
        const int comp[6] = {0, 4, 8, 1, 5, 6};
        for (int c = 0; c < 6; ++c) {
          const double d =
              ((double)Wq[((s - s0) * 9 + comp[c]) * kcs + kl] * iW - w_tar[6 * (size_t)s + c]) *
              ns_inv;
          ev += d * d;
        }
      }
      const double de = (eu - e_tar[s]) * ns_inv;
      double* o = sq + ((size_t)k * S + s) * 3;
      if (eF == kBadScale || eW == kBadScale) {
        o[0] = o[1] = o[2] = __builtin_nan("");
      } else {
        o[0] = de * de;
        o[1] = ef;
        o[2] = ev;
      }
    }
  }
}

template <int CT>
void launch_net(nep_ctx ctx, nep_dataset ds, int n_pop, const float* Z, bool first) {
  launch_kernel(ctx, first, false, k_pop_wfrag, dim3(n_pop), dim3(64), ctx->n_par, Z,
                ds->wfrag.ptr, ds->wb2.ptr, ds->dqbound.ptr);
  const int per_block = 16 * CT * (kBlock / 64);
  launch_kernel(ctx, false, false, k_pop_net<CT>,
                dim3(blocks_for(ds->N, per_block), (n_pop + kNetChunk - 1) / kNetChunk),
                dim3(kBlock), ds->N, n_pop, (const float*)ds->qpad.ptr,
                (const float4*)ds->wfrag.ptr, (const float*)ds->wb2.ptr, ds->dq.ptr, ds->U.ptr);
}

}  // namespace

int population_max_structure() { return kLdsInts / 3 - 3; }

hipError_t prepare_dataset_geometry(nep_ctx ctx, nep_dataset ds) {
  const int N = ds->N, cap = ds->cap, S = ds->S;
  const size_t ncap = (size_t)N * cap;
  hipError_t e = ds->prec.ensure(ncap);
  if (e == hipSuccess) e = ds->pcidx.ensure(ncap);
  if (e == hipSuccess) e = ds->pn_ang.ensure(N);
  if (e == hipSuccess) e = ds->pn_in.ensure(N);
  if (e == hipSuccess) e = ds->desc.ensure((size_t)kDescRow * N);
  if (e == hipSuccess) e = ds->qpad.ensure((size_t)kQ * N);
  if (e == hipSuccess) e = ds->pmeta.ensure(N);
  if (e == hipSuccess) e = ds->stile0.ensure(S);
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
  k_pop_qpad<<<blocks_for((size_t)N * kQ, kBlock), kBlock, 0, st>>>(N, ds->desc.ptr, ds->qpad.ptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // Layout of the contraction operands from the pair counts (host side).
  std::vector<int> n_in(N), n_ang(N);
  if ((e = hipMemcpyAsync(n_in.data(), ds->pn_in.ptr, sizeof(int) * N, hipMemcpyDeviceToHost,
                          st)) != hipSuccess ||
      (e = hipMemcpyAsync(n_ang.data(), ds->pn_ang.ptr, sizeof(int) * N, hipMemcpyDeviceToHost,
                          st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return e;
  std::vector<int4> meta(N);
  size_t chunks = 0, pairs = 0, pairs_a = 0;
  for (int i = 0; i < N; ++i) {
    meta[i] = make_int4((int)chunks, (int)pairs, n_in[i], n_ang[i]);
    chunks += atom_chunks(n_in[i], n_ang[i]);
    pairs += n_in[i];
    pairs_a += n_ang[i];
  }
  ds->pairs_r = (long long)pairs;
  ds->pairs_a = (long long)pairs_a;
  if (chunks >= (1ull << 31) || pairs >= (1ull << 31)) return hipErrorInvalidValue;
  // Tiles: consecutive whole structures whose accumulators fit the LDS for
  // tile_kc individuals: 3 KC (atoms + 3 structures) 32-bit values.
  const std::vector<int>& off = ds->off_host;
  int largest = 0;
  for (int s = 0; s < S; ++s) largest = std::max(largest, off[s + 1] - off[s]);
  const int tile_kc = std::min(64, kLdsInts / (3 * (largest + 3)));
  if (tile_kc < 1) return hipErrorInvalidValue;
  const int units = kLdsInts / (3 * tile_kc);
  // tiles are filled to kTileTarget units (a larger structure takes a tile
  // alone): many small tiles balance the blocks over the compute units
  const int target = std::min(units, kTileTarget);
  std::vector<int> toff{0}, ts0{0}, st0(S);
  int cur = 0;
  for (int s = 0; s < S; ++s) {
    const int ns = off[s + 1] - off[s] + 3;
    if (cur > 0 && cur + ns > target) {
      toff.push_back(off[s]);
      ts0.push_back(s);
      cur = 0;
    }
    st0[s] = toff.back();
    cur += ns;
  }
  toff.push_back(N);
  ts0.push_back(S);
  const int T = (int)ts0.size() - 1;
  std::vector<long long> work(T, 0);
  std::vector<int> deg(T, 1);
  int tile_max = 0;
  for (int t = 0; t < T; ++t) {
    tile_max = std::max(tile_max, toff[t + 1] - toff[t]);
    for (int i = toff[t]; i < toff[t + 1]; ++i) {
      work[t] += atom_chunks(n_in[i], n_ang[i]);
      // a force component receives a radial and an angular part per incoming
      // pair (as many as the receiver's own pairs) and its own force
      deg[t] = std::max(deg[t], 2 * n_in[i] + 1);
    }
  }
  std::vector<int> order(T);
  for (int t = 0; t < T; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return work[a] > work[b]; });
  ds->n_tiles = T;
  ds->tile_max = tile_max;
  ds->tile_kc = tile_kc;
  if ((e = ds->pfrag.ensure((chunks + kPadChunks) * 64)) != hipSuccess ||
      (e = ds->ppair.ensure(pairs + kPadPairs)) != hipSuccess ||
      (e = ds->tile_off.ensure(T + 1)) != hipSuccess ||
      (e = ds->tile_s0.ensure(T + 1)) != hipSuccess ||
      (e = ds->tile_order.ensure(T)) != hipSuccess ||
      (e = ds->tbound.ensure(T)) != hipSuccess || (e = ds->pnorm.ensure(N)) != hipSuccess)
    return e;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  up(ds->pmeta.ptr, meta.data(), sizeof(int4) * N);
  up(ds->tile_off.ptr, toff.data(), sizeof(int) * (T + 1));
  up(ds->tile_s0.ptr, ts0.data(), sizeof(int) * (T + 1));
  up(ds->tile_order.ptr, order.data(), sizeof(int) * T);
  up(ds->stile0.ptr, st0.data(), sizeof(int) * S);
  if (e == hipSuccess)
    e = hipMemsetAsync(ds->pfrag.ptr, 0, sizeof(float) * (chunks + kPadChunks) * 64, st);
  if (e == hipSuccess)
    e = hipMemsetAsync(ds->ppair.ptr + pairs, 0, sizeof(float4) * kPadPairs, st);
  if (e != hipSuccess) return e;
  k_pop_geo<<<blocks_for((size_t)N * 32, kBlock), kBlock, 0, st>>>(
      N, tile_kc, ds->prec.ptr, ds->pmeta.ptr, ds->desc.ptr, ds->struct_of.ptr, ds->stile0.ptr, rcr, rca,
      ds->pfrag.ptr, ds->ppair.ptr);
  k_pop_norms<<<blocks_for(N, 64), 64, 0, st>>>(N, ds->pmeta.ptr, ds->pfrag.ptr, ds->pnorm.ptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // per tile: deg_t max_i (force-row norm) and sum_i (virial-row norm), the
  // factors of the fixed-point bounds (times the bound on |dU/dq|)
  std::vector<float2> pn(N), tb(T);
  if ((e = hipMemcpyAsync(pn.data(), ds->pnorm.ptr, sizeof(float2) * N, hipMemcpyDeviceToHost,
                          st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return e;
  for (int t = 0; t < T; ++t) {
    float fm = 0.f;
    double vs = 0.0;
    for (int i = toff[t]; i < toff[t + 1]; ++i) {
      fm = std::max(fm, pn[i].x);
      vs += pn[i].y;
    }
    // rounded up a little: the products formed on the device round
    tb[t] = make_float2((float)deg[t] * fm * 1.001f, (float)vs * 1.001f);
  }
  up(ds->tbound.ptr, tb.data(), sizeof(float2) * T);
  if (e != hipSuccess) return e;
  // the host vectors above are read by the copies
  return hipStreamSynchronize(st);
}

int population_variants() { return 3; }
int population_atoms(int variant) { return variant == 0 ? 16 : (variant == 1 ? 32 : 64); }

hipError_t launch_population(nep_ctx ctx, nep_dataset ds, int n_pop, const float* Z, int variant,
                             bool first) {
  if (ds->N == 0 || n_pop == 0) return hipSuccess;
  const int KC = ds->tile_kc;
  if (KC < 1 || ds->n_tiles < 1) return hipErrorInvalidConfiguration;
  switch (variant) {
    case 0:
      launch_net<1>(ctx, ds, n_pop, Z, first);
      break;
    case 2:
      launch_net<4>(ctx, ds, n_pop, Z, first);
      break;
    default:
      launch_net<2>(ctx, ds, n_pop, Z, first);
  }
  for (int k0 = 0; k0 < n_pop; k0 += KC)
    launch_kernel(ctx, false, false, k_pop_contract, dim3(ds->n_tiles),
                  dim3(64 * kContractWaves), ds->N, ds->S, k0, std::min(KC, n_pop - k0), KC, n_pop,
                  (const int*)ds->tile_order.ptr, (const int*)ds->tile_off.ptr,
                  (const int*)ds->tile_s0.ptr, (const int*)ds->off.ptr,
                  (const int*)ds->struct_of.ptr, (const int4*)ds->pmeta.ptr,
                  (const float*)ds->pfrag.ptr, (const float4*)ds->ppair.ptr,
                  (const float*)ds->dq.ptr, (const float*)ds->U.ptr,
                  (const float2*)ds->tbound.ptr, (const float*)ds->dqbound.ptr,
                  (const double*)ds->f_tar.ptr,
                  (const double*)ds->e_tar.ptr, (const double*)ds->w_tar.ptr,
                  (const int*)ds->has_v.ptr, ds->struct_sq.ptr);
  return hipGetLastError();
}

}  // namespace nep
