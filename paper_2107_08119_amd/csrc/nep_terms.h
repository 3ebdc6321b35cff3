// Per-pair and per-atom terms of the NEP model shared by the force kernels:
// descriptor accumulation of one pair, the network with its input gradient,
// and the partial force of one pair.
//
// The angular descriptor (Eq. qinl) is used in the factorised form that the
// addition theorem gives (paper, text after Eq. N_des): with real harmonics
// Yhat_lm normalised so that sum_m Yhat_lm(u) Yhat_lm(v) = P_l(u.v),
//   q_nl = sum_j sum_k g_n(r_ij) g_n(r_ik) P_l(cos theta_ijk) = sum_m c_nlm^2,
//   c_nlm = sum_j g_n(r_ij) Yhat_lm(r_ij / r_ij),
// which equals the double sum (j = k terms included) up to rounding.  The
// partial force (Sec. II D) is
//   dU_i/dr_ij = sum_n dU/dq_n g_n'(r) u
//              + sum_lm [ B_lm Yhat_lm(u) u + A_lm (grad Yhat_lm - u (u.grad Yhat_lm)) / r ],
// with a_nlm = 2 dU/dq_nl c_nlm, A_lm = sum_n a_nlm g_n(r), B_lm = sum_n a_nlm g_n'(r).
// Since g_n = f_c (T_n + 1)/2, both come from At_lm = a'_0lm + sum_{n>=1} a_nlm T_n
// (a'_0lm = 2 a_0lm + sum_{n>=1} a_nlm, folded once per atom) and
// D_lm = sum_{n>=1} a_nlm T_n':  A_lm = f_c At_lm / 2,
// B_lm = f_c' At_lm / 2 + f_c (dx/dr) D_lm / 2.
#pragma once

#include "nep_device.h"

namespace nep {

template <int NR, int NA, int LMAX>
struct Model {
  static constexpr int kNLM = (LMAX + 1) * (LMAX + 1) - 1;  // harmonics l = 1..LMAX
  static constexpr int kNDES = NR + NA * LMAX;
};

// Add pair (dx, dy, dz) to the radial sums (when rad) and to the angular
// moments c[NA][NLM] (when ang).  The radial sums are kept as
// R_n = sum_j f_c T_n (R_0 = sum_j f_c); radial_finish turns them into
// q_n = sum_j g_n = (R_n + R_0) / 2 once they are complete.
template <int NR, int NA, int LMAX>
__device__ __forceinline__ void pair_descriptor(float dx, float dy, float dz, bool rad, bool ang,
                                                float rcr_inv, float rca_inv, float* q,
                                                float (&c)[NA][Model<NR, NA, LMAX>::kNLM]) {
  constexpr int NLM = Model<NR, NA, LMAX>::kNLM;
  const float r2 = pair_r2(dx, dy, dz);
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float r = r2 * rinv;
  if (rad) {
    float fc, T[NR];
    chebyshev_values<NR>(r, rcr_inv, fc, T);
    q[0] += fc;
#pragma unroll
    for (int a = 1; a < NR; ++a) q[a] += fc * T[a];
  }
  if (ang) {
    float g[NA];
    radial_basis<NA, false>(r, rca_inv, g, nullptr);
    const float x = dx * rinv, y = dy * rinv, z = dz * rinv;
    const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
    const float xyz = xy * z;
    (void)xyz;
#define NEP_ACC(idx, YV, GX, GY, GZ)                                        \
  if constexpr ((idx) < NLM) {                                              \
    const float yv = (YV);                                                  \
    _Pragma("unroll") for (int a = 0; a < NA; ++a) c[a][idx] += g[a] * yv; \
  }
    NEP_YLM_TABLE(NEP_ACC)
#undef NEP_ACC
  }
}

// The sums of pair_descriptor started from one pair instead of from zero:
// q[0..NR) and c are assigned the pair's terms, weighted 0 where the pair
// is not inside the cutoff (rad, ang false), so a lane whose first work item
// is a dummy pair passes zeros on.  The terms are evaluated for every lane
// (finite for any r > 0).
template <int NR, int NA, int LMAX>
__device__ __forceinline__ void pair_descriptor_first(float dx, float dy, float dz, bool rad,
                                                      bool ang, float rcr_inv, float rca_inv,
                                                      float* q,
                                                      float (&c)[NA][Model<NR, NA, LMAX>::kNLM]) {
  constexpr int NLM = Model<NR, NA, LMAX>::kNLM;
  const float r2 = pair_r2(dx, dy, dz);
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float r = r2 * rinv;
  {
    float fc, T[NR];
    chebyshev_values<NR>(r, rcr_inv, fc, T);
    const float w = rad ? fc : 0.f;
    q[0] = w;
#pragma unroll
    for (int a = 1; a < NR; ++a) q[a] = w * T[a];
  }
  float g[NA];
  radial_basis<NA, false>(r, rca_inv, g, nullptr);
#pragma unroll
  for (int a = 0; a < NA; ++a) g[a] = ang ? g[a] : 0.f;
  const float x = dx * rinv, y = dy * rinv, z = dz * rinv;
  const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  const float xyz = xy * z;
  (void)xyz;
#define NEP_SET(idx, YV, GX, GY, GZ)                                       \
  if constexpr ((idx) < NLM) {                                             \
    const float yv = (YV);                                                 \
    _Pragma("unroll") for (int a = 0; a < NA; ++a) c[a][idx] = g[a] * yv; \
  }
  NEP_YLM_TABLE(NEP_SET)
#undef NEP_SET
}

// q_n = (R_n + R_0) / 2 from the complete sums R_n of pair_descriptor.
template <int NR>
__device__ __forceinline__ void radial_finish(float* q) {
#pragma unroll
  for (int a = 1; a < NR; ++a) q[a] = 0.5f * (q[a] + q[0]);
}

// sum_n dU/dq_n over the radial components, the constant part of
// sum_n dU/dq_n g_n' (pair_force's dq_sum).
template <int NR>
__device__ __forceinline__ float radial_dq_sum(const float* dq) {
  float s = 0.f;
#pragma unroll
  for (int a = 0; a < NR; ++a) s += dq[a];
  return s;
}

// The 24 harmonics Yhat_lm (l = 1..4) of the unit vector (x, y, z).
__device__ __forceinline__ void harmonics(float x, float y, float z, float (&out)[24]) {
  const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  const float xyz = xy * z;
  (void)xyz;
#define NEP_Y(idx, YV, GX, GY, GZ) out[idx] = (YV);
  NEP_YLM_TABLE(NEP_Y)
#undef NEP_Y
}

// Angular components q[NR + n LMAX + l - 1] = sum_m c_nlm^2.
template <int NR, int NA, int LMAX>
__device__ __forceinline__ void angular_invariants(const float (&c)[NA][Model<NR, NA, LMAX>::kNLM],
                                                   float* q) {
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int l = 1; l <= LMAX; ++l) {
      float s2 = 0.f;
#pragma unroll
      for (int m = 0; m < 2 * l + 1; ++m) s2 += c[a][l * l - 1 + m] * c[a][l * l - 1 + m];
      q[NR + a * LMAX + (l - 1)] = s2;
    }
}

// LDS layout of the network: NNEU rows of RS floats (w1 row, b1, w2, padding).
template <int NDES, int NNEU>
struct NetRows {
  static constexpr int RS = nn_row_stride(NDES);
  static constexpr int kFloat4 = NNEU * RS / 4;
};

// Fill the LDS rows from z = [w1 (NNEU x NDES), b1, w2, b2]; returns nothing,
// b2 goes to *b2_out (thread 0).  All threads of the block take part.
template <int NDES, int NNEU>
__device__ __forceinline__ void load_net_rows(const float* __restrict__ z, float4* rows,
                                              float* b2_out) {
  constexpr int RS = NetRows<NDES, NNEU>::RS;
  float* sw = reinterpret_cast<float*>(rows);
  for (int t = threadIdx.x; t < NNEU * RS; t += blockDim.x) {
    const int mu = t / RS, v = t % RS;
    float w = 0.f;
    if (v < NDES)
      w = z[mu * NDES + v];
    else if (v == NDES)
      w = z[NNEU * NDES + mu];
    else if (v == NDES + 1)
      w = z[NNEU * (NDES + 1) + mu];
    sw[t] = w;
  }
  if (threadIdx.x == 0) *b2_out = z[NNEU * (NDES + 2)];
}

// LDS row of one atom in network_mfma: 32 descriptor slots (dU/dq on the
// way back), U at column 32, padding to 36 floats (rows off a multiple of 32
// banks, 16-byte aligned).
constexpr int kNetX = 36;
constexpr int net_rows(int lanes) { return 64 / lanes > 16 ? 64 / lanes : 16; }

// The network (Eqs. nn1, nn2) and dU/dq for the 64 / L atoms of a wave on the
// matrix cores.  x is the wave's LDS block of net_rows(L) rows of kNetX
// floats; all 64 lanes of the wave take part; every lane ends with its
// atom's U and dq.  With H = W1 Q^T (neurons x atoms) and
// G = w2 (1 - tanh^2(H - b1)), dq = W1^T G: each product is a 16x16x4 MFMA
// chain per 16-neuron (forward) or 16-descriptor (backward) tile and 16
// atoms.  Forward K step s takes descriptor 8 (l/16) + s in lane l, so a lane
// reads 8 consecutive descriptors; backward step (t, r) takes neuron
// 16 t + 4 (l/16) + r, which is element r of the lane's forward tile t, so G
// feeds the second product from the registers the first one left it in.
template <int NDES, int NNEU, int L>
__device__ __forceinline__ void network_mfma(const float* q, const float4* rows, float b2,
                                             float* x, float* dq, float& u) {
  static_assert(NDES <= 32 && NNEU <= 32 && NNEU >= 1, "two 16-wide tiles");
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int RS = NetRows<NDES, NNEU>::RS;
  constexpr int AW = 64 / L;                  // atoms of the wave
  constexpr int AT = AW >= 16 ? AW / 16 : 1;  // tiles of 16 atoms
  const float* sw = reinterpret_cast<const float*>(rows);
  const int wl = threadIdx.x & 63, g = wl >> 4, j = wl & 15;
  const int aw = wl / L, sub = wl % L;
  // descriptor in, zero-padded to 32, written by the atom's first lane
  if (sub == 0) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = 4 * t + e < NDES ? q[4 * t + e] : 0.f;
      *reinterpret_cast<float4*>(x + aw * kNetX + 4 * t) = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // forward operands: W1[16 t + j][8 g + s] (rows past NNEU repeat the last
  // row; their output weight is zero below), the lane's b1 and w2
  float af[2][8];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int mu = min(16 * t + j, NNEU - 1);
    const float4 r0 = rows[(mu * RS + 8 * g) / 4], r1 = rows[(mu * RS + 8 * g) / 4 + 1];
    af[t][0] = r0.x, af[t][1] = r0.y, af[t][2] = r0.z, af[t][3] = r0.w;
    af[t][4] = r1.x, af[t][5] = r1.y, af[t][6] = r1.z, af[t][7] = r1.w;
  }
  float gv[AT][2][4];
  float us[AT];
#pragma unroll
  for (int at = 0; at < AT; ++at) {
    const float* xr = x + (16 * at + j) * kNetX + 8 * g;
    const float4 b0 = *reinterpret_cast<const float4*>(xr);
    const float4 b1v = *reinterpret_cast<const float4*>(xr + 4);
    const float bq[8] = {b0.x, b0.y, b0.z, b0.w, b1v.x, b1v.y, b1v.z, b1v.w};
    float up = 0.f;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      f4 h = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 8; ++s) h = __builtin_amdgcn_mfma_f32_16x16x4f32(af[t][s], bq[s], h, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mu = 16 * t + 4 * g + r;
        const int mc = min(mu, NNEU - 1);
        const float w2 = mu < NNEU ? sw[mc * RS + NDES + 1] : 0.f;
        const float act = h[r] - sw[mc * RS + NDES];
        // tanh and its derivative 1 - tanh^2 from e = exp(-2|a|) (no cancellation)
        const float ea = __expf(-2.f * fabsf(act));
        const float inv = __builtin_amdgcn_rcpf(1.f + ea);
        const float th = copysignf((1.f - ea) * inv, act);
        up += w2 * th;
        gv[at][t][r] = w2 * (4.f * ea * inv * inv);
      }
    }
    // sum over the four lane groups (neurons 4 g .. 4 g + 3 of each tile)
    up += __shfl_xor(up, 16, 64);
    up += __shfl_xor(up, 32, 64);
    us[at] = up - b2;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // backward: dq^T[16 d + 4 g + r][atom] into the atom rows, U at column 32
#pragma unroll
  for (int at = 0; at < AT; ++at) {
    float* xr = x + (16 * at + j) * kNetX;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int mc = min(16 * t + 4 * g + r, NNEU - 1);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(sw[mc * RS + 16 * d + j], gv[at][t][r], acc,
                                                     0, 0, 0);
        }
      *reinterpret_cast<float4*>(xr + 16 * d + 4 * g) = make_float4(acc[0], acc[1], acc[2], acc[3]);
    }
    if (g == 0) xr[32] = us[at];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const float4* xo = reinterpret_cast<const float4*>(x + aw * kNetX);
#pragma unroll
  for (int t = 0; t < (NDES + 3) / 4; ++t) {
    const float4 v = xo[t];
    const float e4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (4 * t + e < NDES) dq[4 * t + e] = e4[e];
  }
  u = x[aw * kNetX + 32];
}

// a_nlm = 2 dU/dq_nl c_nlm in place of c, then row 0 replaced by
// a'_0lm = 2 a_0lm + sum_{n>=1} a_nlm (the constant part of sum_n a_nlm (T_n + 1)).
template <int NR, int NA, int LMAX>
__device__ __forceinline__ void angular_coefficients(const float* dq,
                                                     float (&c)[NA][Model<NR, NA, LMAX>::kNLM]) {
  constexpr int NLM = Model<NR, NA, LMAX>::kNLM;
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int l = 1; l <= LMAX; ++l) {
      const float f = 2.f * dq[NR + a * LMAX + (l - 1)];
#pragma unroll
      for (int m = 0; m < 2 * l + 1; ++m) c[a][l * l - 1 + m] *= f;
    }
#pragma unroll
  for (int m = 0; m < NLM; ++m) {
    float s = 2.f * c[0][m];
#pragma unroll
    for (int a = 1; a < NA; ++a) s += c[a][m];
    c[0][m] = s;
  }
}

// Partial force dU_i/dr_ij of pair (dx, dy, dz) from dq (radial part, when
// rad; dq_sum = radial_dq_sum(dq)) and the angular coefficients a as left by
// angular_coefficients (when ang).  Radial part: sum_n dU/dq_n g_n' =
// f_c' (S_1 + dq_sum) / 2 + f_c (dx/dr) S_2 / 2 with S_1 = sum_n dU/dq_n T_n
// and S_2 = sum_n dU/dq_n T_n'.
template <int NR, int NA, int LMAX>
__device__ __forceinline__ void pair_force(float dx, float dy, float dz, bool rad, bool ang,
                                           float rcr_inv, float rca_inv, const float* dq,
                                           float dq_sum,
                                           const float (&c)[NA][Model<NR, NA, LMAX>::kNLM],
                                           float& px, float& py, float& pz) {
  constexpr int NLM = Model<NR, NA, LMAX>::kNLM;
  const float r2 = pair_r2(dx, dy, dz);
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float r = r2 * rinv;
  const float x = dx * rinv, y = dy * rinv, z = dz * rinv;
  px = 0.f;
  py = 0.f;
  pz = 0.f;
  if (rad) {
    float fc, dfc, dxdr, T[NR], dT[NR];
    chebyshev_terms<NR>(r, rcr_inv, fc, dfc, dxdr, T, dT);
    float s1 = dq[0], s2 = 0.f;
#pragma unroll
    for (int a = 1; a < NR; ++a) {
      s1 += dq[a] * T[a];
      s2 += dq[a] * dT[a];
    }
    const float f = 0.5f * (dfc * (s1 + dq_sum) + fc * dxdr * s2);
    px += f * x;
    py += f * y;
    pz += f * z;
  }
  if (ang) {
    float fc, dfc, dxdr, T[NA], dT[NA];
    chebyshev_terms<NA>(r, rca_inv, fc, dfc, dxdr, T, dT);
    const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
    const float xyz = xy * z;
    (void)xyz;
    float sa = 0.f, sd = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
#define NEP_PF(idx, YV, GX, GY, GZ)                   \
  if constexpr ((idx) < NLM) {                        \
    float At = c[0][idx], D = 0.f;                    \
    _Pragma("unroll") for (int a = 1; a < NA; ++a) {  \
      At += c[a][idx] * T[a];                         \
      D += c[a][idx] * dT[a];                         \
    }                                                 \
    sa += At * (YV);                                  \
    sd += D * (YV);                                   \
    gx += At * (GX);                                  \
    gy += At * (GY);                                  \
    gz += At * (GZ);                                  \
  }
    NEP_YLM_TABLE(NEP_PF)
#undef NEP_PF
    const float sb = 0.5f * (dfc * sa + fc * dxdr * sd);
    const float hf = 0.5f * fc;
    gx *= hf;
    gy *= hf;
    gz *= hf;
    const float ug = x * gx + y * gy + z * gz;
    px += sb * x + (gx - x * ug) * rinv;
    py += sb * y + (gy - y * ug) * rinv;
    pz += sb * z + (gz - z * ug) * rinv;
  }
}

}  // namespace nep
