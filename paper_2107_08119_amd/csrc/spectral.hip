// Spectral heat transport on gfx950 (Sec. II B of the paper): the
// virial-velocity correlation K(t) = sum_i <W_i(0) . v_i(t)>_ne of an HNEMD
// run, the spectral conductivity kappa(w) from
//   (2 / T V) int K_mu(t) e^{i w t} dt = sum_nu kappa_mu,nu(w) F_e^nu,
// and its quantum correction kappa(w) x^2 e^x / (e^x - 1)^2, x = hbar w / k_B T
// (the correction of Sec. IV C for disordered materials).
//
// The per-atom virials of the last n_lags samples live in a ring of
// [n_lags][9][N] float32 (caller order).  A sample at time t closes lag k
// with the origin t - k for every k <= min(t, n_lags - 1):
//   K_sum[k] += sum_i W_i(t - k) . v_i(t).
// Block sums are added in block order (no atomics), so the sums are
// reproducible bit for bit.  Averages divide by the number of origins of
// each lag.  K is taken even in t; the transform is windowed (Hann) and uses
// the trapezoid rule over the lags, all in float64.
#include <algorithm>
#include <cmath>
#include <new>

#include "nep_device.h"

struct nep_vvcf_s {
  nep_ctx ctx = nullptr;
  int n = 0;       // atoms
  int lags = 0;    // n_lags
  long long samples = 0;
  nep::DevBuf<float> ring;     // [lags][9][n]
  nep::DevBuf<double> ksum;    // [lags][3]
  nep::DevBuf<double> part;    // [lags][blocks][3]
  nep::DevBuf<double> kavg;    // [lags][3]
  nep::DevBuf<double> nu;      // [n_nu]
  nep::DevBuf<double> kappa;   // [2][3][n_nu]
};

namespace nep {
namespace {

constexpr int kVBlock = 256;   // threads per block
constexpr int kVAtoms = 8;     // atoms per thread

inline unsigned vblocks(int n) {
  return (unsigned)(((size_t)n + (size_t)kVBlock * kVAtoms - 1) / ((size_t)kVBlock * kVAtoms));
}

// Block (b, k): atoms b*kVBlock*kVAtoms + tid + kVBlock*a; lag k reads the
// ring slot of sample t - k.  part[k][b][mu] = sum over its atoms of
// sum_nu W_mu,nu v_nu (float64 products of the float32 virial).
__global__ __launch_bounds__(kVBlock) void k_vvcf_blocks(int n, int lags, int head,
                                                         const float* __restrict__ ring,
                                                         const double* __restrict__ vel,
                                                         double* __restrict__ part) {
  const int b = (int)blockIdx.x, k = (int)blockIdx.y;
  const int slot = (head - k + lags) % lags;
  const float* __restrict__ W = ring + (size_t)slot * 9 * n;
  double acc[3] = {0.0, 0.0, 0.0};
  const int base = b * kVBlock * kVAtoms + (int)threadIdx.x;
#pragma unroll
  for (int a = 0; a < kVAtoms; ++a) {
    const int i = base + a * kVBlock;
    if (i < n) {
      const double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
#pragma unroll
      for (int mu = 0; mu < 3; ++mu)
        acc[mu] += (double)W[(size_t)(3 * mu) * n + i] * vx +
                   (double)W[(size_t)(3 * mu + 1) * n + i] * vy +
                   (double)W[(size_t)(3 * mu + 2) * n + i] * vz;
    }
  }
  __shared__ double sw[kVBlock / 64][3];
  const double s = block_sum<3>(acc, sw);
  if (threadIdx.x < 3) part[((size_t)k * gridDim.x + b) * 3 + threadIdx.x] = s;
}

// Thread (k, mu): ksum[k][mu] += sum over blocks in order.
__global__ void k_vvcf_add(int lags_done, int nblocks, const double* __restrict__ part,
                           double* __restrict__ ksum) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * lags_done) return;
  const int k = t / 3, mu = t % 3;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += part[((size_t)k * nblocks + b) * 3 + mu];
  ksum[t] += s;
}

// Averages over the origins of each lag: lag k has samples - k of them.
__global__ void k_vvcf_average(int lags, long long samples, const double* __restrict__ ksum,
                               double* __restrict__ kavg) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * lags) return;
  const long long cnt = samples - t / 3;
  kavg[t] = cnt > 0 ? ksum[t] / (double)cnt : 0.0;
}

// Thread (mu, f): kappa[0][mu][f] = unit * 2 / (T V F_e) * 2 * dt *
// sum_k c_k K_mu(k) h_k cos(2 pi nu_f t_k), c = 1/2 at both ends, Hann h;
// kappa[1] = kappa[0] * x^2 e^x / (e^x - 1)^2.
__global__ void k_vvcf_spectrum(int lags, int n_nu, const double* __restrict__ kavg,
                                const double* __restrict__ nu, double dt_fs, double pref,
                                double x_per_thz, double* __restrict__ kappa) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * n_nu) return;
  const int mu = t / n_nu, f = t % n_nu;
  const double w = 2.0 * M_PI * nu[f] * dt_fs * 1.0e-3;  // radians per lag
  double s = 0.0;
  for (int k = 0; k < lags; ++k) {
    const double c = (k == 0 || k == lags - 1) ? 0.5 : 1.0;
    const double h = lags == 1 ? 1.0 : 0.5 * (1.0 + cos(M_PI * (double)k / (double)(lags - 1)));
    s += c * kavg[3 * k + mu] * h * cos(w * (double)k);
  }
  const double kap = pref * s;
  kappa[t] = kap;
  const double x = x_per_thz * nu[f];
  double q = 1.0;
  if (x > 0.0) {
    const double em1 = expm1(x);
    q = x * x * (em1 + 1.0) / (em1 * em1);
  }
  kappa[3 * n_nu + t] = kap * q;
}

inline unsigned blocks_of(size_t work, int block) { return (unsigned)((work + block - 1) / block); }

}  // namespace
}  // namespace nep

using namespace nep;

extern "C" {

nep_status nep_vvcf_create(nep_ctx ctx, int n_atoms, int n_lags, nep_vvcf* out) {
  if (!ctx || !out) return NEP_EINVAL;
  *out = nullptr;
  if (n_atoms < 1 || n_atoms > kMaxAtoms) return fail(ctx, NEP_EINVAL, "n_atoms out of range");
  if (n_lags < 1 || n_lags > 65535) return fail(ctx, NEP_EINVAL, "n_lags must be in [1, 65535]");
  if ((double)n_lags * 9.0 * n_atoms * 4.0 > 64.0e9)
    return fail(ctx, NEP_EINVAL, "virial ring above 64 GB");
  DeviceGuard guard(ctx->device);
  nep_vvcf v = new (std::nothrow) nep_vvcf_s();
  if (!v) return fail(ctx, NEP_ENOMEM, "vvcf");
  v->ctx = ctx;
  v->n = n_atoms;
  v->lags = n_lags;
  hipError_t e = v->ring.ensure((size_t)n_lags * 9 * n_atoms);
  if (e == hipSuccess) e = v->ksum.ensure((size_t)3 * n_lags);
  if (e == hipSuccess) e = v->kavg.ensure((size_t)3 * n_lags);
  if (e == hipSuccess) e = v->part.ensure((size_t)3 * n_lags * vblocks(n_atoms));
  if (e == hipSuccess) e = hipMemsetAsync(v->ksum.ptr, 0, sizeof(double) * 3 * n_lags, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    nep_vvcf_destroy(v);
    return check_hip(ctx, e, "allocating the correlation buffers");
  }
  *out = v;
  return NEP_OK;
}

void nep_vvcf_destroy(nep_vvcf v) {
  if (!v) return;
  DeviceGuard guard(v->ctx->device);
  (void)hipStreamSynchronize(v->ctx->stream);
  v->ring.release();
  v->ksum.release();
  v->part.release();
  v->kavg.release();
  v->nu.release();
  v->kappa.release();
  delete v;
}

nep_status nep_vvcf_sample(nep_ctx ctx, nep_vvcf v, const float* W_dev, const double* vel_dev) {
  if (!ctx || !v || v->ctx != ctx) return NEP_EINVAL;
  if (!W_dev || !vel_dev) return fail(ctx, NEP_EINVAL, "W_dev and vel_dev are required");
  DeviceGuard guard(ctx->device);
  const int n = v->n, lags = v->lags;
  const int head = (int)(v->samples % lags);
  hipError_t e = hipMemcpyAsync(v->ring.ptr + (size_t)head * 9 * n, W_dev, sizeof(float) * 9 * n,
                                hipMemcpyDeviceToDevice, ctx->stream);
  if (e != hipSuccess) return check_hip(ctx, e, "copying the virials");
  const int done = (int)std::min<long long>(v->samples + 1, lags);
  const unsigned nb = vblocks(n);
  launch_kernel(ctx, true, false, k_vvcf_blocks, dim3(nb, done), dim3(kVBlock), n, lags, head,
                (const float*)v->ring.ptr, vel_dev, v->part.ptr);
  launch_kernel(ctx, false, true, k_vvcf_add, dim3(blocks_of((size_t)3 * done, 256)), dim3(256),
                done, (int)nb, (const double*)v->part.ptr, v->ksum.ptr);
  e = hipGetLastError();
  if (e != hipSuccess) return check_hip(ctx, e, "launching the correlation kernels");
  ++v->samples;
  return NEP_OK;
}

nep_status nep_vvcf_get(nep_ctx ctx, nep_vvcf v, double* K_host, long long* samples) {
  if (!ctx || !v || v->ctx != ctx) return NEP_EINVAL;
  DeviceGuard guard(ctx->device);
  const int lags = v->lags;
  launch_kernel(ctx, true, true, k_vvcf_average, dim3(blocks_of((size_t)3 * lags, 256)), dim3(256),
                lags, v->samples, (const double*)v->ksum.ptr, v->kavg.ptr);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && K_host)
    e = hipMemcpyAsync(K_host, v->kavg.ptr, sizeof(double) * 3 * lags, hipMemcpyDeviceToHost,
                       ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return check_hip(ctx, e, "reading the correlation");
  if (samples) *samples = v->samples;
  return NEP_OK;
}

nep_status nep_vvcf_spectrum(nep_ctx ctx, nep_vvcf v, double dt_fs, double temperature,
                             double volume, double fe, int n_nu, const double* nu_thz_host,
                             double* kappa_host, double* kappa_q_host) {
  if (!ctx || !v || v->ctx != ctx) return NEP_EINVAL;
  if (!(dt_fs > 0.0) || !(temperature > 0.0) || !(volume > 0.0) || !(fe != 0.0) ||
      !std::isfinite(dt_fs) || !std::isfinite(temperature) || !std::isfinite(volume) ||
      !std::isfinite(fe))
    return fail(ctx, NEP_EINVAL, "dt, T, V must be > 0 and F_e nonzero");
  if (n_nu < 1 || n_nu > (1 << 24) || !nu_thz_host || !kappa_host)
    return fail(ctx, NEP_EINVAL, "n_nu, nu and kappa are required");
  if (v->samples == 0) return fail(ctx, NEP_ESTATE, "no samples yet");
  DeviceGuard guard(ctx->device);
  hipError_t e = v->nu.ensure((size_t)n_nu);
  if (e == hipSuccess) e = v->kappa.ensure((size_t)6 * n_nu);
  if (e == hipSuccess)
    e = hipMemcpyAsync(v->nu.ptr, nu_thz_host, sizeof(double) * n_nu, hipMemcpyHostToDevice,
                       ctx->stream);
  if (e != hipSuccess) return check_hip(ctx, e, "spectrum buffers");
  const int lags = v->lags;
  launch_kernel(ctx, true, false, k_vvcf_average, dim3(blocks_of((size_t)3 * lags, 256)), dim3(256),
                lags, v->samples, (const double*)v->ksum.ptr, v->kavg.ptr);
  // W/(m K THz) per eV/(A K): (1 eV/fs in W) (1/A in 1/m) (1 fs in ps)
  const double unit = 1.602176634e-19 / 1.0e-15 * 1.0e10 * 1.0e-3;
  const double pref = unit * 2.0 / (temperature * volume * fe) * 2.0 * dt_fs;
  // x = hbar 2 pi nu / k_B T with nu in THz
  const double x_per_thz = 1.054571817e-34 * 2.0 * M_PI * 1.0e12 / (1.380649e-23 * temperature);
  launch_kernel(ctx, false, true, k_vvcf_spectrum, dim3(blocks_of((size_t)3 * n_nu, 256)),
                dim3(256), lags, n_nu, (const double*)v->kavg.ptr, (const double*)v->nu.ptr,
                dt_fs, pref, x_per_thz, v->kappa.ptr);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(kappa_host, v->kappa.ptr, sizeof(double) * 3 * n_nu, hipMemcpyDeviceToHost,
                       ctx->stream);
  if (e == hipSuccess && kappa_q_host)
    e = hipMemcpyAsync(kappa_q_host, v->kappa.ptr + (size_t)3 * n_nu, sizeof(double) * 3 * n_nu,
                       hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  return check_hip(ctx, e, "computing the spectrum");
}

}  // extern "C"
