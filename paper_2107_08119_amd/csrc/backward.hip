// Parameter gradient of an energy + force objective over a dataset (gfx950).
//
// For G(z) = sum_s gE_s E_s + sum_i gF_i . F_i, Sec. II A gives
// sum_i gF_i . F_i = -sum_a sum_nu dU_a/dq_nu delta q_a,nu with the
// directional derivative of the descriptor along gF,
//   delta q_a = sum_j (dq_a / dr_aj) . (gF_j - gF_a),
// so that, with x = tanh(a_mu), s = 1 - x^2, t_mu = sum_nu w1[mu][nu] delta q_nu
// and g_a = gE of atom a's structure (Eqs. nn1, nn2):
//   dG/dw1[mu][k] = w2_mu sum_a (alpha_a,mu q_a,k - s_a,mu delta q_a,k),
//   dG/db1[mu]    = -w2_mu sum_a alpha_a,mu,
//   dG/dw2[mu]    = sum_a beta_a,mu,
//   dG/db2        = -sum_a g_a,
// with alpha = s (g + 2 x t) and beta = g x - s t.
//
// k_grad_atoms evaluates q and delta q per atom (lanes split the neighbour
// slots, as in the force kernel; delta q uses the same factorised angular
// form) and writes (alpha, s, beta, q, delta q, g) per atom.  k_grad_blocks
// contracts them over blocks of atoms into float64 partial gradients, and
// k_grad_final adds the blocks in order.
#include "nep_device.h"

namespace nep {
namespace {

inline unsigned blocks_for(size_t work, int block) { return (unsigned)((work + block - 1) / block); }

constexpr int kLanes = 4;
constexpr int kChunk = 64;  // atoms per block in the contraction

template <int NR, int NA, int LMAX, int NNEU>
struct GradLayout {
  static constexpr int NDES = NR + NA * LMAX;
  static constexpr int ALPHA = 0, S = NNEU, BETA = 2 * NNEU, Q = 3 * NNEU, DQ = 3 * NNEU + NDES,
                       G = 3 * NNEU + 2 * NDES, FIELDS = 3 * NNEU + 2 * NDES + 1;
};

template <int idx>
constexpr int l_of() {
  return idx < 3 ? 1 : (idx < 8 ? 2 : (idx < 15 ? 3 : 4));
}

template <int NR, int NA, int LMAX, int NNEU, int L>
__global__ __launch_bounds__(kBlock) void k_grad_atoms(
    int n, const double* __restrict__ pos, const uint32_t* __restrict__ nl,
    const int* __restrict__ cnt_r, const int* __restrict__ cnt_a,
    const double* __restrict__ boxes, const int* __restrict__ struct_of,
    const float* __restrict__ zpar, float rc_r, float rc_a, const double* __restrict__ gE,
    const float* __restrict__ gF, float* __restrict__ rec) {
  using Lay = GradLayout<NR, NA, LMAX, NNEU>;
  constexpr int NLM = (LMAX + 1) * (LMAX + 1) - 1;
  constexpr int NDES = Lay::NDES;
  constexpr int NPAR = (NDES + 2) * NNEU + 1;
  __shared__ float sz[NPAR];
  for (int t = threadIdx.x; t < NPAR; t += blockDim.x) sz[t] = zpar[t];
  __syncthreads();
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gid / L;
  const int lane = gid % L;
  const bool active = i < n;
  const int ii = active ? i : 0;
  const int cr = active ? cnt_r[i] : 0;
  const int ca = active ? cnt_a[i] : 0;
  const double xi = pos[ii], yi = pos[n + ii], zi = pos[2 * n + ii];
  const double* H = boxes + 9 * (size_t)struct_of[ii];
  const float rcr_inv = 1.f / rc_r, rca_inv = 1.f / rc_a;

  float q[NDES];
  float c[NA][NLM];
#pragma unroll
  for (int v = 0; v < NDES; ++v) q[v] = 0.f;
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int m = 0; m < NLM; ++m) c[a][m] = 0.f;
  for (int s = lane; s < cr; s += L) {
    int j;
    float dx, dy, dz;
    displacement(nl[(size_t)s * n + i], pos, n, xi, yi, zi, H, j, dx, dy, dz);
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * rinv;
    if (r < rc_r) {
      float g[NR];
      radial_basis<NR, false>(r, rcr_inv, g, nullptr);
#pragma unroll
      for (int a = 0; a < NR; ++a) q[a] += g[a];
    }
    if (s < ca && r < rc_a) {
      float g[NA];
      radial_basis<NA, false>(r, rca_inv, g, nullptr);
      const float x = dx * rinv, y = dy * rinv, z = dz * rinv;
      const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
      const float xyz = xy * z;
      (void)xyz;
#define NEP_ACC(idx, YV, GX, GY, GZ)                                         \
  if constexpr ((idx) < NLM) {                                               \
    const float yv = (YV);                                                   \
    _Pragma("unroll") for (int a = 0; a < NA; ++a) c[a][idx] += g[a] * yv;   \
  }
      NEP_YLM_TABLE(NEP_ACC)
#undef NEP_ACC
    }
  }
#pragma unroll
  for (int a = 0; a < NR; ++a) q[a] = group_sum<L>(q[a]);
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int m = 0; m < NLM; ++m) c[a][m] = group_sum<L>(c[a][m]);
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int l = 1; l <= LMAX; ++l) {
      float s2 = 0.f;
#pragma unroll
      for (int m = 0; m < 2 * l + 1; ++m) s2 += c[a][l * l - 1 + m] * c[a][l * l - 1 + m];
      q[NR + a * LMAX + (l - 1)] = s2;
    }

  // delta q: directional derivative of the descriptor along gF
  float dq[NDES];
#pragma unroll
  for (int v = 0; v < NDES; ++v) dq[v] = 0.f;
  if (gF) {
    const float gxi = gF[ii], gyi = gF[n + ii], gzi = gF[2 * n + ii];
    for (int s = lane; s < cr; s += L) {
      int j;
      float dx, dy, dz;
      displacement(nl[(size_t)s * n + i], pos, n, xi, yi, zi, H, j, dx, dy, dz);
      const float r2 = dx * dx + dy * dy + dz * dz;
      const float rinv = __builtin_amdgcn_rsqf(r2);
      const float r = r2 * rinv;
      const float x = dx * rinv, y = dy * rinv, z = dz * rinv;
      const float Dx = gF[j] - gxi, Dy = gF[n + j] - gyi, Dz = gF[2 * n + j] - gzi;
      const float uD = x * Dx + y * Dy + z * Dz;
      if (r < rc_r) {
        float g[NR], dg[NR];
        radial_basis<NR, true>(r, rcr_inv, g, dg);
#pragma unroll
        for (int a = 0; a < NR; ++a) dq[a] += dg[a] * uD;
      }
      if (s < ca && r < rc_a) {
        float g[NA], dg[NA];
        radial_basis<NA, true>(r, rca_inv, g, dg);
        const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
        const float xyz = xy * z;
        (void)xyz;
        // d q_nl = sum_m 2 c_nlm [g_n' Y_lm (u.D) + g_n (grad Y_lm . D - (u.grad Y_lm)(u.D)) / r]
#define NEP_JVP(idx, YV, GX, GY, GZ)                                                     \
  if constexpr ((idx) < NLM) {                                                           \
    const float gxv = (GX), gyv = (GY), gzv = (GZ);                                      \
    const float yd = (YV) * uD;                                                          \
    const float gd = (gxv * Dx + gyv * Dy + gzv * Dz - (x * gxv + y * gyv + z * gzv) * uD) * rinv; \
    _Pragma("unroll") for (int a = 0; a < NA; ++a)                                       \
      dq[NR + a * LMAX + (l_of<idx>() - 1)] += 2.f * c[a][idx] * (dg[a] * yd + g[a] * gd); \
  }
        NEP_YLM_TABLE(NEP_JVP)
#undef NEP_JVP
      }
    }
#pragma unroll
    for (int v = 0; v < NDES; ++v) dq[v] = group_sum<L>(dq[v]);
  }

  // network quantities per neuron (neurons split over the lanes)
  const float* w1 = sz;
  const float* b1 = sz + NNEU * NDES;
  const float ga = (active && gE) ? (float)gE[struct_of[i]] : 0.f;
  if (active) {
    for (int mu = lane; mu < NNEU; mu += L) {
      float act = -b1[mu], t = 0.f;
#pragma unroll
      for (int v = 0; v < NDES; ++v) {
        act += w1[mu * NDES + v] * q[v];
        t += w1[mu * NDES + v] * dq[v];
      }
      const float ea = __expf(-2.f * fabsf(act));
      const float inv = __builtin_amdgcn_rcpf(1.f + ea);
      const float xm = copysignf((1.f - ea) * inv, act);
      const float sm = 4.f * ea * inv * inv;
      rec[(size_t)(Lay::ALPHA + mu) * n + i] = sm * (ga + 2.f * xm * t);
      rec[(size_t)(Lay::S + mu) * n + i] = sm;
      rec[(size_t)(Lay::BETA + mu) * n + i] = ga * xm - sm * t;
    }
    for (int v = lane; v < NDES; v += L) {
      rec[(size_t)(Lay::Q + v) * n + i] = q[v];
      rec[(size_t)(Lay::DQ + v) * n + i] = dq[v];
    }
    if (lane == 0) rec[(size_t)Lay::G * n + i] = ga;
  }
}

// Block b contracts atoms [b*kChunk, (b+1)*kChunk) into out[b][N_par] (float64).
template <int NR, int NA, int LMAX, int NNEU>
__global__ __launch_bounds__(kBlock) void k_grad_blocks(int n, const float* __restrict__ rec,
                                                         const float* __restrict__ zpar,
                                                         double* __restrict__ out) {
  using Lay = GradLayout<NR, NA, LMAX, NNEU>;
  constexpr int NDES = Lay::NDES;
  constexpr int NPAR = (NDES + 2) * NNEU + 1;
  __shared__ float sr[Lay::FIELDS][kChunk];
  const int a0 = blockIdx.x * kChunk;
  const int na = min(kChunk, n - a0);
  for (int t = threadIdx.x; t < Lay::FIELDS * kChunk; t += blockDim.x) {
    const int f = t / kChunk, a = t % kChunk;
    sr[f][a] = a < na ? rec[(size_t)f * n + a0 + a] : 0.f;
  }
  __syncthreads();
  const float* w2 = zpar + NNEU * NDES + NNEU;
  for (int p = threadIdx.x; p < NPAR; p += blockDim.x) {
    double acc = 0.0;
    if (p < NNEU * NDES) {
      const int mu = p / NDES, k = p % NDES;
      for (int a = 0; a < na; ++a)
        acc += (double)(sr[Lay::ALPHA + mu][a] * sr[Lay::Q + k][a] -
                        sr[Lay::S + mu][a] * sr[Lay::DQ + k][a]);
      acc *= (double)w2[mu];
    } else if (p < NNEU * NDES + NNEU) {
      const int mu = p - NNEU * NDES;
      for (int a = 0; a < na; ++a) acc += (double)sr[Lay::ALPHA + mu][a];
      acc *= -(double)w2[mu];
    } else if (p < NNEU * NDES + 2 * NNEU) {
      const int mu = p - NNEU * NDES - NNEU;
      for (int a = 0; a < na; ++a) acc += (double)sr[Lay::BETA + mu][a];
    } else {
      for (int a = 0; a < na; ++a) acc -= (double)sr[Lay::G][a];
    }
    out[(size_t)blockIdx.x * NPAR + p] = acc;
  }
}

__global__ void k_grad_final(int nblocks, int npar, const double* __restrict__ part,
                             double* __restrict__ grad, float* __restrict__ grad32) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npar) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * npar + p];
  grad[p] = s;
  if (grad32) grad32[p] = (float)s;
}

__global__ void k_grad_positions(int n, const int* __restrict__ struct_of,
                                 const double* __restrict__ gE, const float* __restrict__ F,
                                 double* __restrict__ gpos) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * n) return;
  const int i = t % n;
  gpos[t] = gE ? -gE[struct_of[i]] * (double)F[t] : 0.0;
}

}  // namespace

hipError_t launch_backward(nep_ctx ctx, nep_dataset ds, const float* z, const double* gE,
                           const float* gF, const float* F, double* gpos, double* grad,
                           float* grad32) {
  using Lay = GradLayout<9, 5, 4, 30>;
  const int N = ds->N;
  constexpr int NPAR = (Lay::NDES + 2) * 30 + 1;
  const unsigned nblk = blocks_for((size_t)N, kChunk);
  hipError_t e = ds->grad_rec.ensure((size_t)Lay::FIELDS * N);
  if (e == hipSuccess) e = ds->grad_part.ensure((size_t)nblk * NPAR);
  if (e != hipSuccess) return e;
  launch_kernel(ctx, true, false, k_grad_atoms<9, 5, 4, 30, kLanes>,
                dim3(blocks_for((size_t)N * kLanes, kBlock)), dim3(kBlock), N,
                (const double*)ds->pos.ptr, (const uint32_t*)ds->nl.ptr, (const int*)ds->cnt_r.ptr,
                (const int*)ds->cnt_a.ptr, (const double*)ds->boxes.ptr,
                (const int*)ds->struct_of.ptr, z, (float)ctx->hyper.rc_radial,
                (float)ctx->hyper.rc_angular, gE, gF, ds->grad_rec.ptr);
  launch_kernel(ctx, false, false, k_grad_blocks<9, 5, 4, 30>, dim3(nblk), dim3(kBlock), N,
                (const float*)ds->grad_rec.ptr, z, ds->grad_part.ptr);
  launch_kernel(ctx, false, gpos == nullptr, k_grad_final, dim3(blocks_for(NPAR, kBlock)),
                dim3(kBlock), (int)nblk, NPAR, (const double*)ds->grad_part.ptr, grad, grad32);
  if (gpos)
    launch_kernel(ctx, false, true, k_grad_positions, dim3(blocks_for((size_t)3 * N, kBlock)),
                  dim3(kBlock), N, (const int*)ds->struct_of.ptr, gE, F, gpos);
  return hipGetLastError();
}

}  // namespace nep
