// Pass 1 for any model size within n_max^R, n_max^A <= 15, l_max <= 4 and
// at most 64 hidden neurons (the paper's models of Sec. III, e.g. 80-50-1):
// one 64-lane wave per atom, lanes over the atom's neighbour pairs.
//
// The terms are those of nep_terms.h (factorised angular descriptor, network,
// partial force of Sec. II D), with the per-atom sums done by the wave:
//   * radial q_n: each lane adds f_c T_n of its pairs, then a fixed-order
//     wave sum gives R_n and q_n = (R_n + R_0)/2 (g_n = f_c (T_n + 1)/2);
//   * angular moments c_nlm = sum_j g_n(r_ij) Yhat_lm(u_ij): the lanes write
//     their pairs' g_n and Yhat_lm to LDS and lane k accumulates outputs
//     (n, lm) = k, k + 64, ... over the pairs in index order;
//   * network: lane mu evaluates neuron mu; dU/dq_v is formed by lane v from
//     the neurons' w2 sech^2 in LDS;
//   * partial forces: lane p evaluates pair p from dU/dq and a_nlm in LDS,
//     as sums over T_n and T_n' (the n = 0 terms folded per atom), and
//     stores the pair vector r_ij in the atom's own slot for pass 2 (systems
//     of up to kPairVectorMaxAtoms atoms).
// Every sum has a fixed order, so results are reproducible bit for bit.
//
// Multicomponent systems take the descriptor and the hidden layer's input in
// float64 (pair geometry, basis, harmonics, the sums q and c_nlm, and the
// pre-activations with tanh and sech^2): the pair weights sqrt(Z_i Z_j) (up to
// 82) scale the descriptor up by about two orders, unscaled input weights then
// put pre-activations in the hundreds, and sech^2 there changes relatively by
// twice any absolute error of the pre-activation, which float32 sums make about
// 1e-5.  The partial forces stay float32.
#include <type_traits>

#include "nep_terms.h"

namespace nep {
namespace {

// Largest sizes of the runtime-sized instantiation.
constexpr int kMaxR = 16, kMaxA = 16, kMaxNeu = 64;
constexpr int kWaves = 4;  // atoms per block

// Sizes of one instantiation: TR > 0 fixes (n_max^R + 1, n_max^A + 1, l_max,
// N_neu) = (TR, TA, TL, TNEU) at compile time (loops unrolled, LDS sized to
// the model); TR == 0 takes them at run time up to the maxima above.
template <int TR, int TA, int TL, int TNEU>
struct Shape {
  static constexpr bool kFixed = TR > 0;
  static constexpr int MR = kFixed ? TR : kMaxR;
  static constexpr int MA = kFixed ? TA : kMaxA;
  static constexpr int ML = kFixed ? TL : 4;
  static constexpr int MLM = (ML + 1) * (ML + 1) - 1;
  static constexpr int MNEU = kFixed ? TNEU : kMaxNeu;
  static constexpr int MDES = MR + MA * ML;
};

// Sum over the 64 lanes of a wave in a fixed order; every lane gets the
// same bits (each step adds two partial sums, which commutes exactly).
__device__ __forceinline__ float wave_sum(float v) {
  v = group_sum<16>(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Fixed-order sum over the 64 lanes in float64 (butterfly: each step adds the
// same two values on both partners, so every lane gets the same bits).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// r_ij of list entry e in float64, rounded exactly as the float32
// displacement is before its final rounding (so the two agree to float32).
__device__ __forceinline__ void displacement_d(uint32_t e, const double* __restrict__ pos, int n,
                                               double xi, double yi, double zi, const double* h,
                                               int& j, double& dx, double& dy, double& dz) {
  j = (int)(e & kAtomMask);
  int n0, n1, n2;
  unpack_image(e, n0, n1, n2);
  const double a0 = (double)n0, a1 = (double)n1, a2 = (double)n2;
  dx = (pos[j] - xi) + (a0 * h[0] + a1 * h[3] + a2 * h[6]);
  dy = (pos[n + j] - yi) + (a0 * h[1] + a1 * h[4] + a2 * h[7]);
  dz = (pos[2 * n + j] - zi) + (a0 * h[2] + a1 * h[5] + a2 * h[8]);
}

constexpr double kPiD = 3.14159265358979323846;

// cos(pi t) for t near [0, 1] as -sin(y), y = pi (t - 1/2), from the Taylor
// series of sin through y^21 (for |y| <= pi/2 the first omitted term is below
// 2e-18, under float64 rounding).
__device__ __forceinline__ double cos_pi_unit(double t) {
  const double y = kPiD * (t - 0.5);
  const double y2 = y * y;
  double p = 1.0 / 51090942171709440000.0;  // 1/21!
  p = p * y2 - 1.0 / 121645100408832000.0;  // 1/19!
  p = p * y2 + 1.0 / 355687428096000.0;     // 1/17!
  p = p * y2 - 1.0 / 1307674368000.0;       // 1/15!
  p = p * y2 + 1.0 / 6227020800.0;          // 1/13!
  p = p * y2 - 1.0 / 39916800.0;            // 1/11!
  p = p * y2 + 1.0 / 362880.0;              // 1/9!
  p = p * y2 - 1.0 / 5040.0;                // 1/7!
  p = p * y2 + 1.0 / 120.0;                 // 1/5!
  p = p * y2 - 1.0 / 6.0;                   // 1/3!
  p = p * y2 + 1.0;
  return -y * p;
}

// f_c(r) = (1 + cos(pi r/r_c))/2 and T_n(x), x = 2 (r/r_c - 1)^2 - 1, n < NB,
// in float64: the factors of g_n = f_c (T_n + 1)/2 (Eq. g_n).
template <int NB>
__device__ __forceinline__ void chebyshev_values_d(double r, double rc_inv, double& fc, double* T) {
  const double t = r * rc_inv;
  fc = 0.5 * (1.0 + cos_pi_unit(t));
  const double tm1 = t - 1.0;
  const double x = 2.0 * tm1 * tm1 - 1.0;
  T[0] = 1.0;
  if constexpr (NB > 1) T[1] = x;
#pragma unroll
  for (int k = 2; k < NB; ++k) T[k] = 2.0 * x * T[k - 1] - T[k - 2];
}

// g_n(r), n < nb (<= MB), zero beyond, in float64.
template <int MB>
__device__ __forceinline__ void radial_basis_d(double r, double rc_inv, int nb, double* g) {
  double fc, T[MB];
  chebyshev_values_d<MB>(r, rc_inv, fc, T);
#pragma unroll
  for (int k = 0; k < MB; ++k) g[k] = k < nb ? 0.5 * (T[k] + 1.0) * fc : 0.0;
}

// The 24 harmonics Yhat_lm (l = 1..4) in float64: the same polynomials, with
// the square roots in their float64 values.
#pragma push_macro("NEP_S3")
#pragma push_macro("NEP_S5")
#pragma push_macro("NEP_S6")
#pragma push_macro("NEP_S10")
#pragma push_macro("NEP_S15")
#pragma push_macro("NEP_S35")
#pragma push_macro("NEP_S70")
#undef NEP_S3
#undef NEP_S5
#undef NEP_S6
#undef NEP_S10
#undef NEP_S15
#undef NEP_S35
#undef NEP_S70
#define NEP_S3 1.7320508075688772935
#define NEP_S5 2.2360679774997896964
#define NEP_S6 2.4494897427831780982
#define NEP_S10 3.1622776601683793320
#define NEP_S15 3.8729833462074168852
#define NEP_S35 5.9160797830996160426
#define NEP_S70 8.3666002653407554798
__device__ __forceinline__ void harmonics_d(double x, double y, double z, double (&out)[24]) {
  const double xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  const double xyz = xy * z;
  (void)xyz;
#define NEP_Y(idx, YV, GX, GY, GZ) out[idx] = (YV);
  NEP_YLM_TABLE(NEP_Y)
#undef NEP_Y
}
#pragma pop_macro("NEP_S70")
#pragma pop_macro("NEP_S35")
#pragma pop_macro("NEP_S15")
#pragma pop_macro("NEP_S10")
#pragma pop_macro("NEP_S6")
#pragma pop_macro("NEP_S5")
#pragma pop_macro("NEP_S3")

// Radial basis g_n, n < nb (<= MB), and optionally g_n'.
template <int MB>
__device__ __forceinline__ void radial_basis_n(float r, float rc_inv, int nb, float* g, float* dg) {
  float gg[MB], dd[MB];
  radial_basis<MB, true>(r, rc_inv, gg, dd);
#pragma unroll
  for (int n = 0; n < MB; ++n) {
    g[n] = n < nb ? gg[n] : 0.f;
    if (dg) dg[n] = n < nb ? dd[n] : 0.f;
  }
}

// F64: the float64 descriptor and hidden-layer input of multicomponent
// systems (wspd = sqrt(Z) in float64 beside wsp).
template <int TR, int TA, int TL, int TNEU, bool F64>
__global__ __launch_bounds__(64 * kWaves) void k_partials_generic(
    int n, const double* __restrict__ pos, const uint32_t* __restrict__ nl,
    const int* __restrict__ cnt_r, const int* __restrict__ cnt_a, const int* __restrict__ rev,
    Box box, const float* __restrict__ z, int nr_rt, int na_rt, int lmax_rt, int nneu_rt,
    double rc_rd, double rc_ad, const float* __restrict__ wsp,
    const double* __restrict__ wspd, const int* __restrict__ perm,
    Partial3* __restrict__ pin, float* __restrict__ fown, float* __restrict__ U,
    Partial3* __restrict__ geo) {
  using S = Shape<TR, TA, TL, TNEU>;
  using DT = typename std::conditional<F64, double, float>::type;
  const float rc_r = (float)rc_rd, rc_a = (float)rc_ad;
  constexpr int kMaxR = S::MR, kMaxA = S::MA, kMaxLM = S::MLM, kMaxNeu = S::MNEU;
  constexpr int kMaxDes = S::MDES;
  const int NR = S::kFixed ? TR : nr_rt;
  const int NA = S::kFixed ? TA : na_rt;
  const int LMAX = S::kFixed ? TL : lmax_rt;
  const int NNEU = S::kFixed ? TNEU : nneu_rt;
  const int NLM = (LMAX + 1) * (LMAX + 1) - 1;
  const int NDES = NR + NA * LMAX;
  // Compiled shapes with l_max = 4 read LDS four floats at a time: the
  // network rows, the descriptor and the neurons' w2 sech^2 are padded with
  // zeros to multiples of 4, and the harmonics rows hold 24 floats.
  constexpr bool kVec = S::kFixed && TL == 4 && !F64;
  constexpr int kDes4 = ((kMaxDes + 3) / 4) * 4;
  constexpr int kRS = kVec ? kDes4 + (kDes4 % 32 == 0 ? 4 : 0) : kMaxDes + 1;
  constexpr int kNeuRows = kVec ? ((kMaxNeu + 3) / 4) * 4 : kMaxNeu;
  constexpr int kYS = kVec ? kMaxLM : kMaxLM + 1;
  const int RS = kVec ? kRS : NDES + 1;  // LDS row of neuron mu: w1[mu][:] (padded)
  __shared__ __align__(16) float s_w1[kNeuRows * kRS];
  __shared__ float s_b1[kMaxNeu], s_w2[kMaxNeu];
  // pairs staged per round: all 64 lanes' pairs, or in float64 two halves of
  // 32 (half the LDS, so that more waves fit a CU; the sums keep pair order)
  constexpr int kStage = F64 ? 32 : 64;
  __shared__ DT s_g[kWaves][kStage][kMaxA + 1];           // angular g_n of the staged pairs
  __shared__ __align__(16) DT s_y[kWaves][kStage][kYS];   // Yhat_lm of the staged pairs
  __shared__ __align__(16) DT s_q[kWaves][kDes4];
  __shared__ float s_dq[kWaves][kMaxDes];
  __shared__ float s_c[kWaves][kMaxA * kMaxLM];  // c_nlm (float32 path), then a_nlm
  __shared__ double s_cd[F64 ? kWaves : 1][F64 ? kMaxA * kMaxLM : 1];  // c_nlm in float64
  __shared__ __align__(16) float s_gmu[kWaves][kNeuRows];
  if constexpr (kVec) {
    for (int t = threadIdx.x; t < kNeuRows * kRS; t += blockDim.x) {
      const int mu = t / kRS, v = t % kRS;
      s_w1[t] = mu < NNEU && v < NDES ? z[mu * NDES + v] : 0.f;
    }
  } else {
    for (int t = threadIdx.x; t < NNEU * NDES; t += blockDim.x)
      s_w1[(t / NDES) * RS + t % NDES] = z[t];
  }
  for (int t = threadIdx.x; t < NNEU; t += blockDim.x) {
    s_b1[t] = z[NNEU * NDES + t];
    s_w2[t] = z[NNEU * (NDES + 1) + t];
  }
  const float b2 = z[NNEU * (NDES + 2)];
  __syncthreads();

  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int i = (int)xcd_block(blockIdx.x, gridDim.x) * kWaves + wave;
  if (i >= n) return;  // whole waves leave together; no block barrier below
  const int cr = cnt_r[i], ca = cnt_a[i];
  const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
  // multicomponent weight of pair (i, j): sqrt(Z_i) sqrt(Z_j), 1 for one species
  const float wi = wsp ? wsp[perm[i]] : 1.f;
  const float rcr_inv = 1.f / rc_r, rca_inv = 1.f / rc_a;
  const double rcr_inv_d = 1.0 / rc_rd, rca_inv_d = 1.0 / rc_ad;
  const float rcr2 = rc_r * rc_r, rca2 = rc_a * rc_a;
  const int nout = NA * NLM;  // angular moments, lane k owns k, k + 64, ...
  DT qr[kMaxR];
  constexpr int kR4 = (kMaxA * 6 + 63) / 64;  // rounds of the four-output groups
  DT cacc[kVec ? 1 : (kMaxA * kMaxLM + 63) / 64];
  float4 cacc4[kVec ? kR4 : 1];
#pragma unroll
  for (int a = 0; a < kMaxR; ++a) qr[a] = 0;
#pragma unroll
  for (int r = 0; r < (kVec ? 1 : (kMaxA * kMaxLM + 63) / 64); ++r) cacc[r] = 0;
#pragma unroll
  for (int r = 0; r < (kVec ? kR4 : 1); ++r) cacc4[r] = make_float4(0.f, 0.f, 0.f, 0.f);
  auto wave_lds_sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };

  // ---- descriptor
  for (int base = 0; base < cr; base += 64) {
    const int s = base + lane;
    DT g[kMaxA], yh[kMaxLM];
#pragma unroll
    for (int a = 0; a < kMaxA; ++a) g[a] = 0;
#pragma unroll
    for (int m = 0; m < kMaxLM; ++m) yh[m] = 0;
    if (s < cr) {
      int j;
      float dx, dy, dz;
      if constexpr (F64) {
        double ex, ey, ez;
        displacement_d(nl[(size_t)s * n + i], pos, n, xi, yi, zi, box.h, j, ex, ey, ez);
        dx = (float)ex;
        dy = (float)ey;
        dz = (float)ez;
        // in or out of a cutoff exactly as the float32 partial-force loop decides
        const float r2 = pair_r2(dx, dy, dz);
        const double wij = wspd[perm[i]] * wspd[perm[j]];
        const double r = sqrt(ex * ex + ey * ey + ez * ez);
        if (r2 < rcr2) {
          double fc, T[kMaxR];
          chebyshev_values_d<kMaxR>(r, rcr_inv_d, fc, T);
          const double wf = wij * fc;
          qr[0] += wf;
#pragma unroll
          for (int a = 1; a < kMaxR; ++a) qr[a] += wf * T[a];
        }
        if (s < ca && r2 < rca2) {
          radial_basis_d<kMaxA>(r, rca_inv_d, NA, g);
#pragma unroll
          for (int a = 0; a < kMaxA; ++a) g[a] *= wij;
          const double rinv = 1.0 / r;
          harmonics_d(ex * rinv, ey * rinv, ez * rinv, yh);
        }
      } else {
        displacement(nl[(size_t)s * n + i], pos, n, xi, yi, zi, box.h, j, dx, dy, dz);
        const float wij = wsp ? wi * wsp[perm[j]] : 1.f;
        const float r2 = pair_r2(dx, dy, dz);
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float r = r2 * rinv;
        if (r2 < rcr2) {  // entries a >= NR are never read
          float fc, T[kMaxR];
          chebyshev_values<kMaxR>(r, rcr_inv, fc, T);
          const float wf = wij * fc;
          qr[0] += wf;
#pragma unroll
          for (int a = 1; a < kMaxR; ++a) qr[a] += wf * T[a];
        }
        if (s < ca && r2 < rca2) {
          radial_basis_n<kMaxA>(r, rca_inv, NA, g, nullptr);
#pragma unroll
          for (int a = 0; a < kMaxA; ++a) g[a] *= wij;
          harmonics(dx * rinv, dy * rinv, dz * rinv, yh);
        }
      }
    }
    for (int half = 0; half < 64 / kStage; ++half) {
    if (lane / kStage == half) {
#pragma unroll
      for (int a = 0; a < kMaxA; ++a) s_g[wave][lane % kStage][a] = g[a];
#pragma unroll
      for (int m = 0; m < kMaxLM; ++m) s_y[wave][lane % kStage][m] = yh[m];
    }
    wave_lds_sync();
    // pairs past the list's angular part have g = 0: skip them
    const int np = max(0, min(kStage, min(cr, ca) - base - half * kStage));
    if constexpr (kVec) {  // lane k owns outputs (n, 4 m4 .. 4 m4 + 3), k = 6 n + m4
#pragma unroll
      for (int r = 0; r < kR4; ++r) {
        const int k = lane + 64 * r;
        if (k < NA * 6) {
          const int a = k / 6, m4 = k % 6;
          float4 acc = cacc4[r];
          for (int p = 0; p < np; ++p) {
            const float gv = s_g[wave][p][a];
            const float4 y4 = *reinterpret_cast<const float4*>(&s_y[wave][p][4 * m4]);
            acc.x += gv * y4.x;
            acc.y += gv * y4.y;
            acc.z += gv * y4.z;
            acc.w += gv * y4.w;
          }
          cacc4[r] = acc;
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < (kMaxA * kMaxLM + 63) / 64; ++r) {
        const int k = lane + 64 * r;
        if (k < nout) {
          const int a = k / NLM, m = k % NLM;
          DT acc = cacc[r];
          for (int p = 0; p < np; ++p) acc += s_g[wave][p][a] * s_y[wave][p][m];
          cacc[r] = acc;
        }
      }
    }
    wave_lds_sync();
    }
  }
  // radial components q_0 = R_0, q_n = (R_n + R_0)/2, and angular moments to LDS
  const DT r0 = wave_sum(qr[0]);
  if (lane == 0) s_q[wave][0] = r0;
#pragma unroll
  for (int a = 1; a < kMaxR; ++a) {
    const DT v = wave_sum(qr[a]);
    if (lane == 0 && a < NR) s_q[wave][a] = (DT)0.5 * (v + r0);
  }
  if constexpr (kVec) {
#pragma unroll
    for (int r = 0; r < kR4; ++r) {
      const int k = lane + 64 * r;
      if (k < NA * 6) {
        s_c[wave][4 * k] = cacc4[r].x;  // (n, 4 m4 + c) is n 24 + 4 m4 + c = 4 k + c
        s_c[wave][4 * k + 1] = cacc4[r].y;
        s_c[wave][4 * k + 2] = cacc4[r].z;
        s_c[wave][4 * k + 3] = cacc4[r].w;
      }
    }
    for (int v = NDES + lane; v < kDes4; v += 64) s_q[wave][v] = 0.f;  // padding
  } else {
#pragma unroll
    for (int r = 0; r < (kMaxA * kMaxLM + 63) / 64; ++r) {
      const int k = lane + 64 * r;
      if (k < nout) {
        if constexpr (F64)
          s_cd[wave][k] = cacc[r];
        else
          s_c[wave][k] = cacc[r];
      }
    }
  }
  wave_lds_sync();
  // angular components q_nl = sum_m c_nlm^2
  if (lane < NA * LMAX) {
    const int a = lane / LMAX, l = lane % LMAX + 1;
    DT s2 = 0;
    for (int m = 0; m < 2 * l + 1; ++m) {
      const int k = a * NLM + l * l - 1 + m;
      const DT v = F64 ? (DT)s_cd[F64 ? wave : 0][F64 ? k : 0] : (DT)s_c[wave][k];
      s2 += v * v;
    }
    s_q[wave][NR + a * LMAX + (l - 1)] = s2;
  }
  wave_lds_sync();

  // ---- network (Eqs. nn1, nn2): lane mu is neuron mu
  DT u = 0;
  if (lane < NNEU) {
    DT act = -(DT)s_b1[lane];
    if constexpr (kVec) {
#pragma unroll 4
      for (int v4 = 0; v4 < kDes4 / 4; ++v4) {
        const float4 w4 = *reinterpret_cast<const float4*>(&s_w1[lane * kRS + 4 * v4]);
        const float4 q4 = *reinterpret_cast<const float4*>(&s_q[wave][4 * v4]);
        act += w4.x * q4.x;
        act += w4.y * q4.y;
        act += w4.z * q4.z;
        act += w4.w * q4.w;
      }
    } else {
      for (int v = 0; v < NDES; ++v) act += (DT)s_w1[lane * RS + v] * s_q[wave][v];
    }
    if constexpr (F64) {
      const double ea = exp(-2.0 * fabs(act));
      const double inv = 1.0 / (1.0 + ea);
      const double th = copysign((1.0 - ea) * inv, act);
      u = (double)s_w2[lane] * th;
      s_gmu[wave][lane] = (float)((double)s_w2[lane] * (4.0 * ea * inv * inv));
    } else {
      const float ea = __expf(-2.f * fabsf(act));
      const float inv = __builtin_amdgcn_rcpf(1.f + ea);
      const float th = copysignf((1.f - ea) * inv, act);
      u = s_w2[lane] * th;
      s_gmu[wave][lane] = s_w2[lane] * (4.f * ea * inv * inv);
    }
  } else if (kVec && lane < kNeuRows) {
    s_gmu[wave][lane] = 0.f;  // padding (its w1 row is zero too)
  }
  u = wave_sum(u) - (DT)b2;
  if (lane == 0) U[i] = (float)u;
  wave_lds_sync();
  // dU/dq_v: lane v (two rounds for up to 128 descriptor components)
  for (int v = lane; v < NDES; v += 64) {
    float d = 0.f;
    if constexpr (kVec) {
#pragma unroll 2
      for (int m4 = 0; m4 < kNeuRows / 4; ++m4) {
        const float4 g4 = *reinterpret_cast<const float4*>(&s_gmu[wave][4 * m4]);
        d += g4.x * s_w1[(4 * m4) * kRS + v];
        d += g4.y * s_w1[(4 * m4 + 1) * kRS + v];
        d += g4.z * s_w1[(4 * m4 + 2) * kRS + v];
        d += g4.w * s_w1[(4 * m4 + 3) * kRS + v];
      }
    } else {
      for (int mu = 0; mu < NNEU; ++mu) d += s_gmu[wave][mu] * s_w1[mu * RS + v];
    }
    s_dq[wave][v] = d;
  }
  wave_lds_sync();
  // a_nlm = 2 dU/dq_nl c_nlm
#pragma unroll
  for (int r = 0; r < (kMaxA * kMaxLM + 63) / 64; ++r) {
    const int k = lane + 64 * r;
    if (k < nout) {
      const int a = k / NLM, m = k % NLM;
      int l = 1;
      while ((l + 1) * (l + 1) - 1 <= m) ++l;
      if constexpr (F64)
        s_c[wave][k] = (float)(2.0 * (double)s_dq[wave][NR + a * LMAX + (l - 1)] *
                               s_cd[F64 ? wave : 0][F64 ? k : 0]);
      else
        s_c[wave][k] = 2.f * s_dq[wave][NR + a * LMAX + (l - 1)] * s_c[wave][k];
    }
  }
  wave_lds_sync();
  // row 0 becomes a'_0lm = 2 a_0lm + sum_{n>=1} a_nlm, the constant part of
  // sum_n a_nlm (T_n + 1)
  if (lane < NLM) {
    float s0 = 2.f * s_c[wave][lane];
    for (int a = 1; a < NA; ++a) s0 += s_c[wave][a * NLM + lane];
    s_c[wave][lane] = s0;
  }
  // sum_n dU/dq_n over the radial components
  float dqs = 0.f;
  for (int a = 0; a < NR; ++a) dqs += s_dq[wave][a];
  wave_lds_sync();

  // ---- partial forces: lane p is pair p
  float fx = 0.f, fy = 0.f, fz = 0.f;
  for (int base = 0; base < cr; base += 64) {
    const int s = base + lane;
    if (s < cr) {
      const size_t idx = (size_t)s * n + i;
      int j;
      float dx, dy, dz;
      displacement(nl[idx], pos, n, xi, yi, zi, box.h, j, dx, dy, dz);
      if (geo) geo[idx] = Partial3{dx, dy, dz};  // r_ij for pass 2's virial
      const int dst = rev[idx] * n + j;
      const float r2 = pair_r2(dx, dy, dz);
      const float rinv = __builtin_amdgcn_rsqf(r2);
      const float r = r2 * rinv;
      const float x = dx * rinv, y = dy * rinv, z = dz * rinv;
      float px = 0.f, py = 0.f, pz = 0.f;
      if (r2 < rcr2) {
        // sum_n dU/dq_n g_n' = f_c' (S_1 + sum_n dU/dq_n)/2 + f_c (dx/dr) S_2/2
        float fc, dfc, dxdr, T[kMaxR], dT[kMaxR];
        chebyshev_terms<kMaxR>(r, rcr_inv, fc, dfc, dxdr, T, dT);
        float s1 = s_dq[wave][0], s2 = 0.f;
#pragma unroll
        for (int a = 1; a < kMaxR; ++a)
          if (a < NR) {
            s1 += s_dq[wave][a] * T[a];
            s2 += s_dq[wave][a] * dT[a];
          }
        const float f = 0.5f * (dfc * (s1 + dqs) + fc * dxdr * s2);
        px += f * x;
        py += f * y;
        pz += f * z;
      }
      if (s < ca && r2 < rca2) {
        float fc, dfc, dxdr, T[kMaxA], dT[kMaxA];
        chebyshev_terms<kMaxA>(r, rca_inv, fc, dfc, dxdr, T, dT);
        const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
        const float xyz = xy * z;
        (void)xyz;
        // per lm: At = a'_0 + sum_{n>=1} a_n T_n, D = sum_{n>=1} a_n T_n';
        // A = f_c At/2 multiplies the harmonic's gradient and
        // B = f_c' At/2 + f_c (dx/dr) D/2 the harmonic
        float st = 0.f, sd = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
        const float* aw = s_c[wave];
#define NEP_PF(idx, YV, GX, GY, GZ)                     \
  if ((idx) < NLM) {                                    \
    float At = aw[(idx)], D = 0.f;                      \
    for (int a = 1; a < NA; ++a) {                      \
      const float c = aw[a * NLM + (idx)];              \
      At += c * T[a];                                   \
      D += c * dT[a];                                   \
    }                                                   \
    st += At * (YV);                                    \
    sd += D * (YV);                                     \
    gx += At * (GX);                                    \
    gy += At * (GY);                                    \
    gz += At * (GZ);                                    \
  }
        NEP_YLM_TABLE(NEP_PF)
#undef NEP_PF
        const float hf = 0.5f * fc;
        const float sb = 0.5f * (dfc * st + fc * dxdr * sd);
        gx *= hf;
        gy *= hf;
        gz *= hf;
        const float ug = x * gx + y * gy + z * gz;
        px += sb * x + (gx - x * ug) * rinv;
        py += sb * y + (gy - y * ug) * rinv;
        pz += sb * z + (gz - z * ug) * rinv;
      }
      if (wsp) {  // every term of the pair carries its weight once
        const float wij = wi * wsp[perm[j]];
        px *= wij;
        py *= wij;
        pz *= wij;
      }
      fx += px;
      fy += py;
      fz += pz;
      pin[(size_t)(unsigned)dst] = Partial3{px, py, pz};
    }
  }
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  fz = wave_sum(fz);
  if (lane == 0) {
    fown[i] = fx;
    fown[n + i] = fy;
    fown[2 * n + i] = fz;
  }
}

inline unsigned blocks_for(size_t work, int block) { return (unsigned)((work + block - 1) / block); }

}  // namespace

bool generic_supports(const nep_hyper& h) {
  return h.n_max_radial + 1 <= kMaxR && h.n_max_angular + 1 <= kMaxA && h.l_max >= 1 &&
         h.l_max <= 4 && h.n_neuron <= kMaxNeu;
}

namespace {

template <int TR, int TA, int TL, int TNEU, bool F64>
void launch_shape(nep_ctx ctx, const double* pos) {
  const System& s = ctx->sys;
  const nep_hyper& h = ctx->hyper;
  const bool species = ctx->species_on();
  launch_kernel(ctx, true, true, k_partials_generic<TR, TA, TL, TNEU, F64>,
                dim3(blocks_for(s.n, kWaves)), dim3(64 * kWaves), s.n, pos,
                (const uint32_t*)s.nl.ptr, (const int*)s.cnt_r.ptr, (const int*)s.cnt_a.ptr,
                (const int*)s.rev.ptr, s.box, (const float*)ctx->z.ptr, h.n_max_radial + 1,
                h.n_max_angular + 1, h.l_max, h.n_neuron, h.rc_radial, h.rc_angular,
                species ? (const float*)ctx->species_w.ptr : (const float*)nullptr,
                species ? (const double*)ctx->species_wd.ptr : (const double*)nullptr,
                (const int*)s.perm.ptr, ctx->p.ptr, ctx->fown.ptr, ctx->U.ptr,
                s.n <= kPairVectorMaxAtoms ? ctx->geo.ptr : (Partial3*)nullptr);
}

bool is_shape(const nep_hyper& h, int nr, int na, int lmax, int nneu) {
  return h.n_max_radial + 1 == nr && h.n_max_angular + 1 == na && h.l_max == lmax &&
         h.n_neuron == nneu;
}

}  // namespace

// Compile-time sizes for the models of Table I (general Si, silicene, PbTe)
// and the default model; every other size takes the runtime-sized kernel.
// Multicomponent systems take the float64-descriptor kernels (compiled sizes
// for the PbTe and default models).
hipError_t launch_partials_generic(nep_ctx ctx, const double* pos) {
  if (ctx->sys.n == 0) return hipSuccess;
  const nep_hyper& h = ctx->hyper;
  if (ctx->species_on()) {
    if (is_shape(h, 13, 7, 4, 40))
      launch_shape<13, 7, 4, 40, true>(ctx, pos);
    else if (is_shape(h, 9, 5, 4, 30))
      launch_shape<9, 5, 4, 30, true>(ctx, pos);
    else
      launch_shape<0, 0, 0, 0, true>(ctx, pos);
  } else if (is_shape(h, 16, 16, 4, 50)) {
    launch_shape<16, 16, 4, 50, false>(ctx, pos);
  } else if (is_shape(h, 13, 13, 4, 40)) {
    launch_shape<13, 13, 4, 40, false>(ctx, pos);
  } else if (is_shape(h, 13, 7, 4, 40)) {
    launch_shape<13, 7, 4, 40, false>(ctx, pos);
  } else if (is_shape(h, 9, 5, 4, 30)) {
    launch_shape<9, 5, 4, 30, false>(ctx, pos);
  } else {
    launch_shape<0, 0, 0, 0, false>(ctx, pos);
  }
  return hipGetLastError();
}

}  // namespace nep
