// Device helpers shared by the force and population kernels (gfx950).
#pragma once

#include "nep_internal.h"

namespace nep {

constexpr int kBlock = 256;
constexpr float kPi = 3.14159265358979323846f;

// ------------------------------------------------------ XCD-aware blocks
// Workgroups are dispatched to the 8 XCDs of the chip in turn (block b to XCD
// b mod 8), and every XCD has its own L2.  xcd_block maps the dispatch index
// b of nb blocks to a logical block so that each XCD gets one contiguous
// range of logical blocks (a bijection for any nb): neighbouring atoms, whose
// positions and partial-force slots the blocks share, then meet in one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned q = nb / kXcds, rem = nb % kXcds;
  const unsigned x = b % kXcds, r = b / kXcds;
  return x < rem ? x * (q + 1) + r : rem * (q + 1) + (x - rem) * q + r;
}

// ----------------------------------------------------------- lane groups
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

// Sum over aligned groups of L consecutive lanes; every lane gets the sum.
// quad_perm [1,0,3,2] and [2,3,0,1] pair lanes within quads, row_half_mirror
// pairs the two quads of an 8-lane half row, row_mirror the two halves of a row.
template <int L>
__device__ __forceinline__ float group_sum(float v) {
  static_assert(L == 1 || L == 2 || L == 4 || L == 8 || L == 16, "group size");
  if constexpr (L >= 2) v += dpp<0xB1>(v);
  if constexpr (L >= 4) v += dpp<0x4E>(v);
  if constexpr (L >= 8) v += dpp<0x141>(v);
  if constexpr (L >= 16) v += dpp<0x140>(v);
  return v;
}

// ------------------------------------------------------------ radial basis
// sin y and cos y for |y| <= pi/2 from their Taylor series through y^13 and
// y^14 (truncation below 1e-9, under float32 rounding).
__device__ __forceinline__ void sincos_quarter_turn(float y, float& s, float& c) {
  const float y2 = y * y;
  s = y * (1.f + y2 * (-1.f / 6.f +
                       y2 * (1.f / 120.f +
                             y2 * (-1.f / 5040.f +
                                   y2 * (1.f / 362880.f +
                                         y2 * (-1.f / 39916800.f + y2 * (1.f / 6227020800.f)))))));
  c = 1.f + y2 * (-0.5f +
                  y2 * (1.f / 24.f +
                        y2 * (-1.f / 720.f +
                              y2 * (1.f / 40320.f +
                                    y2 * (-1.f / 3628800.f +
                                          y2 * (1.f / 479001600.f + y2 * (-1.f / 87178291200.f)))))));
}

// g_n(r) = (T_n(x) + 1)/2 f_c(r), x = 2 (r/r_c - 1)^2 - 1, n = 0..NB-1 (Eq. g_n),
// with f_c = (1 + cos(pi r/r_c))/2; and g_n'(r) via dT_n/dx = n U_{n-1}(x)
// (Appendix A).  Requires r < r_c.
template <int NB, bool DERIV>
__device__ __forceinline__ void radial_basis(float r, float rc_inv, float* g, float* dg) {
  const float t = r * rc_inv;
  float sy, cy;
  sincos_quarter_turn(kPi * (t - 0.5f), sy, cy);  // cos(pi t) = -sin(pi (t - 1/2))
  const float fc = 0.5f * (1.f - sy);
  const float dfc = -0.5f * kPi * rc_inv * cy;  // -(pi/2r_c) sin(pi t)
  const float tm1 = t - 1.f;
  const float x = 2.f * tm1 * tm1 - 1.f;
  const float dxdr = 4.f * tm1 * rc_inv;
  float T[NB], U[NB];
  T[0] = 1.f;
  U[0] = 1.f;
  if constexpr (NB > 1) {
    T[1] = x;
    U[1] = 2.f * x;
  }
#pragma unroll
  for (int n = 2; n < NB; ++n) {
    T[n] = 2.f * x * T[n - 1] - T[n - 2];
    U[n] = 2.f * x * U[n - 1] - U[n - 2];
  }
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    const float h = 0.5f * (T[n] + 1.f);
    g[n] = h * fc;
    if constexpr (DERIV) {
      const float dT = n == 0 ? 0.f : (float)n * U[n - 1];
      dg[n] = 0.5f * dT * dxdr * fc + h * dfc;
    }
  }
}

// f_c(r) and T_n(x) for n < NB (T_0 = 1), the factors of g_n = f_c (T_n + 1)/2.
template <int NB>
__device__ __forceinline__ void chebyshev_values(float r, float rc_inv, float& fc, float* T) {
  const float t = r * rc_inv;
  float sy, cy;
  sincos_quarter_turn(kPi * (t - 0.5f), sy, cy);
  (void)cy;
  fc = 0.5f * (1.f - sy);
  const float tm1 = t - 1.f;
  const float x = 2.f * tm1 * tm1 - 1.f;
  T[0] = 1.f;
  if constexpr (NB > 1) T[1] = x;
#pragma unroll
  for (int n = 2; n < NB; ++n) T[n] = 2.f * x * T[n - 1] - T[n - 2];
}

// The pieces of g_n and g_n' without the products: T_n(x), dT_n/dx = n U_{n-1}(x)
// for n = 1..NB-1 (entry 0 unused), f_c, f_c' and dx/dr, so that
//   g_n = f_c (T_n + 1) / 2,  g_n' = f_c' (T_n + 1) / 2 + f_c (dx/dr) T_n' / 2.
template <int NB>
__device__ __forceinline__ void chebyshev_terms(float r, float rc_inv, float& fc, float& dfc,
                                                float& dxdr, float* T, float* dT) {
  const float t = r * rc_inv;
  float sy, cy;
  sincos_quarter_turn(kPi * (t - 0.5f), sy, cy);
  fc = 0.5f * (1.f - sy);
  dfc = -0.5f * kPi * rc_inv * cy;
  const float tm1 = t - 1.f;
  const float x = 2.f * tm1 * tm1 - 1.f;
  dxdr = 4.f * tm1 * rc_inv;
  float U[NB];
  T[0] = 1.f;
  U[0] = 1.f;
  dT[0] = 0.f;
  if constexpr (NB > 1) {
    T[1] = x;
    U[1] = 2.f * x;
    dT[1] = 1.f;
  }
#pragma unroll
  for (int n = 2; n < NB; ++n) {
    T[n] = 2.f * x * T[n - 1] - T[n - 2];
    U[n] = 2.f * x * U[n - 1] - U[n - 2];
    dT[n] = (float)n * U[n - 1];
  }
}

// ------------------------------------------------------- angular harmonics
// Real harmonics for l = 1..4 scaled by sqrt(4 pi/(2l+1)) so that
// sum_m Y_lm(u) Y_lm(v) = P_l(u.v) for unit u, v, written as polynomials in
// (x, y, z) = u together with their gradients in R^3.  Entry idx = l^2-1+(m+l).
#define NEP_S3 1.7320508075688772f
#define NEP_S5 2.2360679774997897f
#define NEP_S6 2.4494897427831781f
#define NEP_S10 3.1622776601683795f
#define NEP_S15 3.8729833462074170f
#define NEP_S35 5.9160797830996160f
#define NEP_S70 8.3666002653407555f
#define NEP_YLM_TABLE(X)                                                                        \
  X(0, x, 1.f, 0.f, 0.f)                                                                        \
  X(1, y, 0.f, 1.f, 0.f)                                                                        \
  X(2, z, 0.f, 0.f, 1.f)                                                                        \
  X(3, NEP_S3 * xy, NEP_S3 * y, NEP_S3 * x, 0.f)                                                \
  X(4, NEP_S3 * yz, 0.f, NEP_S3 * z, NEP_S3 * y)                                                \
  X(5, 0.5f * (3.f * zz - 1.f), 0.f, 0.f, 3.f * z)                                              \
  X(6, NEP_S3 * xz, NEP_S3 * z, 0.f, NEP_S3 * x)                                                \
  X(7, 0.5f * NEP_S3 * (xx - yy), NEP_S3 * x, -NEP_S3 * y, 0.f)                                 \
  X(8, 0.25f * NEP_S10 * y * (3.f * xx - yy), 1.5f * NEP_S10 * xy, 0.75f * NEP_S10 * (xx - yy), \
    0.f)                                                                                        \
  X(9, NEP_S15 * xyz, NEP_S15 * yz, NEP_S15 * xz, NEP_S15 * xy)                                 \
  X(10, 0.25f * NEP_S6 * y * (5.f * zz - 1.f), 0.f, 0.25f * NEP_S6 * (5.f * zz - 1.f),          \
    2.5f * NEP_S6 * yz)                                                                         \
  X(11, 0.5f * z * (5.f * zz - 3.f), 0.f, 0.f, 0.5f * (15.f * zz - 3.f))                        \
  X(12, 0.25f * NEP_S6 * x * (5.f * zz - 1.f), 0.25f * NEP_S6 * (5.f * zz - 1.f), 0.f,          \
    2.5f * NEP_S6 * xz)                                                                         \
  X(13, 0.5f * NEP_S15 * z * (xx - yy), NEP_S15 * xz, -NEP_S15 * yz,                            \
    0.5f * NEP_S15 * (xx - yy))                                                                 \
  X(14, 0.25f * NEP_S10 * x * (xx - 3.f * yy), 0.75f * NEP_S10 * (xx - yy),                     \
    -1.5f * NEP_S10 * xy, 0.f)                                                                  \
  X(15, 0.5f * NEP_S35 * xy * (xx - yy), 0.5f * NEP_S35 * y * (3.f * xx - yy),                  \
    0.5f * NEP_S35 * x * (xx - 3.f * yy), 0.f)                                                  \
  X(16, 0.25f * NEP_S70 * yz * (3.f * xx - yy), 1.5f * NEP_S70 * xyz,                           \
    0.75f * NEP_S70 * z * (xx - yy), 0.25f * NEP_S70 * y * (3.f * xx - yy))                     \
  X(17, 0.5f * NEP_S5 * xy * (7.f * zz - 1.f), 0.5f * NEP_S5 * y * (7.f * zz - 1.f),            \
    0.5f * NEP_S5 * x * (7.f * zz - 1.f), 7.f * NEP_S5 * xyz)                                   \
  X(18, 0.25f * NEP_S10 * yz * (7.f * zz - 3.f), 0.f, 0.25f * NEP_S10 * z * (7.f * zz - 3.f),   \
    0.25f * NEP_S10 * y * (21.f * zz - 3.f))                                                    \
  X(19, 0.125f * (35.f * zz * zz - 30.f * zz + 3.f), 0.f, 0.f, 0.125f * z * (140.f * zz - 60.f)) \
  X(20, 0.25f * NEP_S10 * xz * (7.f * zz - 3.f), 0.25f * NEP_S10 * z * (7.f * zz - 3.f), 0.f,   \
    0.25f * NEP_S10 * x * (21.f * zz - 3.f))                                                    \
  X(21, 0.25f * NEP_S5 * (xx - yy) * (7.f * zz - 1.f), 0.5f * NEP_S5 * x * (7.f * zz - 1.f),    \
    -0.5f * NEP_S5 * y * (7.f * zz - 1.f), 3.5f * NEP_S5 * z * (xx - yy))                       \
  X(22, 0.25f * NEP_S70 * xz * (xx - 3.f * yy), 0.75f * NEP_S70 * z * (xx - yy),                \
    -1.5f * NEP_S70 * xyz, 0.25f * NEP_S70 * x * (xx - 3.f * yy))                               \
  X(23, 0.125f * NEP_S35 * (xx * xx - 6.f * xx * yy + yy * yy),                                 \
    0.5f * NEP_S35 * x * (xx - 3.f * yy), 0.5f * NEP_S35 * y * (yy - 3.f * xx), 0.f)

// r_ij = r_j + n.H - r_i formed in float64 from r_j = (xj, yj, zj) and the
// image code of list entry e, rounded to float32; h holds the cell vectors as
// rows.
__device__ __forceinline__ void image_displacement(uint32_t e, double xj, double yj, double zj,
                                                   double xi, double yi, double zi,
                                                   const double* h, float& dx, float& dy,
                                                   float& dz) {
  int n0, n1, n2;
  unpack_image(e, n0, n1, n2);
  const double a0 = (double)n0, a1 = (double)n1, a2 = (double)n2;
  dx = (float)((xj - xi) + (a0 * h[0] + a1 * h[3] + a2 * h[6]));
  dy = (float)((yj - yi) + (a0 * h[1] + a1 * h[4] + a2 * h[7]));
  dz = (float)((zj - zi) + (a0 * h[2] + a1 * h[5] + a2 * h[8]));
}

// The same for list entry e of atom (xi, yi, zi), reading r_j from pos [3][n].
__device__ __forceinline__ void displacement(uint32_t e, const double* __restrict__ pos, int n,
                                             double xi, double yi, double zi, const double* h,
                                             int& j, float& dx, float& dy, float& dz) {
  j = (int)(e & kAtomMask);
  image_displacement(e, pos[j], pos[n + j], pos[2 * n + j], xi, yi, zi, h, dx, dy, dz);
}

// |r_ij|^2 of a float32 displacement with a fixed rounding sequence, so that
// the pair (i, j) and its reverse (j, i), whose displacements are exact
// negatives of each other, are classified alike by every kernel.
__device__ __forceinline__ float pair_r2(float dx, float dy, float dz) {
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// LDS row of one hidden neuron: its N_des input weights, bias, output weight,
// padded to a multiple of 4 floats and off a multiple of 32 (no bank aliasing
// between the rows that the lanes of a group read together).
constexpr int nn_row_stride(int ndes) {
  return ((ndes + 2 + 3) / 4) * 4 + ((((ndes + 2 + 3) / 4) * 4) % 32 == 0 ? 4 : 0);
}

// |r_j + n.H - r_i|^2 evaluated in float64 in the order nep.h documents for
// the neighbour predicate (no fused multiply-add), h = cell vectors as rows.
__device__ __forceinline__ double list_r2(double xj, double yj, double zj, double xi, double yi,
                                          double zi, int n0, int n1, int n2, const double* h) {
#pragma clang fp contract(off)
  const double a0 = (double)n0, a1 = (double)n1, a2 = (double)n2;
  const double dx = (xj - xi) + ((a0 * h[0] + a1 * h[3]) + a2 * h[6]);
  const double dy = (yj - yi) + ((a0 * h[1] + a1 * h[4]) + a2 * h[7]);
  const double dz = (zj - zi) + ((a0 * h[2] + a1 * h[5]) + a2 * h[8]);
  return (dx * dx + dy * dy) + dz * dz;
}

// The lattice shift n.H of list_r2 alone (same operation order), and the
// squared distance from a precomputed shift: list_r2_shifted(.., image_shift(n))
// equals list_r2(.., n) bit for bit.
__device__ __forceinline__ void image_shift(int n0, int n1, int n2, const double* h, double& sx,
                                            double& sy, double& sz) {
#pragma clang fp contract(off)
  const double a0 = (double)n0, a1 = (double)n1, a2 = (double)n2;
  sx = (a0 * h[0] + a1 * h[3]) + a2 * h[6];
  sy = (a0 * h[1] + a1 * h[4]) + a2 * h[7];
  sz = (a0 * h[2] + a1 * h[5]) + a2 * h[8];
}

__device__ __forceinline__ double list_r2_shifted(double xj, double yj, double zj, double xi,
                                                  double yi, double zi, double sx, double sy,
                                                  double sz) {
#pragma clang fp contract(off)
  const double dx = (xj - xi) + sx;
  const double dy = (yj - yi) + sy;
  const double dz = (zj - zi) + sz;
  return (dx * dx + dy * dy) + dz * dz;
}

// Sum of NQ doubles over a block in a fixed order: shuffle tree inside each
// wave, then waves in index order.  The result is valid in threads < NQ
// (thread q holds quantity q).
template <int NQ>
__device__ __forceinline__ double block_sum(double (&v)[NQ], double (&sw)[kBlock / 64][NQ]) {
#pragma unroll
  for (int q = 0; q < NQ; ++q)
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off, 64);
  const int wave = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) sw[wave][q] = v[q];
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < NQ)
    for (int w = 0; w < kBlock / 64; ++w) s += sw[w][threadIdx.x];
  return s;
}

}  // namespace nep
