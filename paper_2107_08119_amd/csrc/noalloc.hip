// nep_evaluate_static: neighbour list and one force evaluation (the work of
// nep_build_neighbors followed by nep_compute) for callers that cannot
// allocate device memory.  Every buffer beyond the caller's inputs and
// outputs is carved from one file-scope device array of fixed size; the call
// makes no hipMalloc or hipFree.
#include <mutex>

#include "nep_internal.h"

namespace nep {
namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;  // 32 MiB per device
constexpr int kMaxDevices = 64;

// The workspace.  Host code never names it past set-up: its host-side name
// is a stand-in, not a device address; the per-device address comes from
// hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};
hipError_t g_status[kMaxDevices] = {};

// Carves aligned sub-ranges off the workspace into DevBuf views.
struct Carver {
  char* base;
  size_t off = 0;
  bool ok = true;
  template <class T>
  void take(DevBuf<T>& b, size_t count) {
    const size_t bytes = ((count > 0 ? count : 1) * sizeof(T) + 255) & ~(size_t)255;
    if (!ok || off + bytes > kScratchBytes) {
      ok = false;
      return;
    }
    b.set_view(base ? reinterpret_cast<T*>(base + off) : nullptr, count > 0 ? count : 1);
    off += bytes;
  }
};

// Views of the list and evaluation buffers for n atoms with cap slots.
// With base == nullptr only the size is worked out.
bool carve(char* base, const System& geo, int n, int cap, System& s, nep_ctx_s& c,
           size_t* used) {
  Carver k{base};
  const size_t ncap = (size_t)n * cap;
  const size_t n3 = (size_t)3 * n;
  k.take(s.nl, ncap);
  k.take(s.rev, ncap);
  k.take(s.cnt_r, n);
  k.take(s.cnt_a, n);
  k.take(s.iperm, n);
  k.take(s.wrap, n3);
  k.take(s.pos_s, n3);
  k.take(s.pos_t, n3);
  k.take(s.vel_s, n3);
  k.take(s.perm, n);
  k.take(s.pos_ref, n3);
  if (geo.use_cells) {
    const size_t ncell = (size_t)geo.nc[0] * geo.nc[1] * geo.nc[2];
    k.take(s.nl_rm, ncap);
    k.take(s.cell_of, n);
    k.take(s.cell_cnt, ncell);
    k.take(s.scan_part, 1024);
    k.take(s.cell_start, ncell + 1);
    k.take(s.cell_fill, ncell);
    k.take(s.cell_atoms, n);
    k.take(s.cell_rec, n);
    k.take(s.vel_t, n3);
    k.take(s.perm_t, n);
    k.take(s.wrap_t, n3);
    k.take(s.cell_t, n);
  }
  k.take(c.p, ncap);
  k.take(c.geo, ncap);
  k.take(c.U, n);
  k.take(c.fown, n3);
  k.take(c.F, n3);
  k.take(c.W, (size_t)9 * n);
  k.take(c.J, n3);
  k.take(c.partials, gather_blocks(n) * 16 + 16);
  *used = k.off;
  return k.ok;
}

// The context's own system, buffers and species, put back on every return.
struct Swap {
  nep_ctx ctx;
  System sys;
  DevBuf<Partial3> p, geo;
  DevBuf<float> U, fown, F, W, J;
  DevBuf<double> partials;
  int species_n;
  bool have_masses;
  explicit Swap(nep_ctx c)
      : ctx(c), sys(c->sys), p(c->p), geo(c->geo), U(c->U), fown(c->fown), F(c->F), W(c->W),
        J(c->J), partials(c->partials), species_n(c->species_n), have_masses(c->have_masses) {}
  ~Swap() {
    ctx->sys = sys;
    ctx->p = p;
    ctx->geo = geo;
    ctx->U = U;
    ctx->fown = fown;
    ctx->F = F;
    ctx->W = W;
    ctx->J = J;
    ctx->partials = partials;
    ctx->species_n = species_n;
    ctx->have_masses = have_masses;
  }
};

}  // namespace

// Once per device, with that device current (nep_create): the device address
// of the workspace.  A failure is kept and reported by nep_evaluate_static.
void scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_status[device] = e;
  if (e == hipSuccess) g_scratch[device] = ptr;
}

}  // namespace nep

using namespace nep;

extern "C" {

size_t nep_static_workspace_bytes(void) { return kScratchBytes; }

nep_status nep_evaluate_static(nep_ctx ctx, int n_atoms, const double* pos_dev,
                               const double* box_host, double skin, int max_neighbors,
                               const double* vel_dev, float* U_dev, float* F_dev, float* W_dev,
                               float* J_dev, double* totals_dev) {
  if (!ctx) return NEP_EINVAL;
  if (!ctx->have_params) return fail(ctx, NEP_ESTATE, "nep_load_params must come first");
  if (n_atoms < 0 || n_atoms > kMaxAtoms)
    return fail(ctx, NEP_EINVAL, "n_atoms must be in [0, 2^23)");
  if (n_atoms > 0 && (!pos_dev || !F_dev))
    return fail(ctx, NEP_EINVAL, "pos_dev and F_dev are required");
  if (J_dev && !vel_dev) return fail(ctx, NEP_EINVAL, "J_dev needs vel_dev");
  if (max_neighbors < 1 || (size_t)max_neighbors * (size_t)(n_atoms > 0 ? n_atoms : 1) >= (1ull << 31))
    return fail(ctx, NEP_EINVAL, "need 1 <= max_neighbors and max_neighbors * n_atoms < 2^31");
  System geo;
  nep_status st = check_box(ctx, box_host, skin, geo);
  if (st != NEP_OK) return st;
  System view;
  nep_ctx_s sizing;
  size_t need = 0;
  if (!carve(nullptr, geo, n_atoms, max_neighbors, view, sizing, &need))
    return fail(ctx, NEP_EINVAL,
                "system needs more than the " + std::to_string(kScratchBytes >> 20) +
                    " MiB static workspace (fewer atoms, fewer max_neighbors or a smaller box "
                    "per atom)");
  DeviceGuard guard(ctx->device);
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) {
      base = g_scratch[ctx->device];
      if (!base) return check_hip(ctx, g_status[ctx->device] != hipSuccess
                                           ? g_status[ctx->device]
                                           : hipErrorNotInitialized,
                                  "locating the static workspace");
    }
  }
  if (!base) return fail(ctx, NEP_EDEVICE, "device index beyond the static workspace table");
  Swap keep(ctx);
  carve(static_cast<char*>(base), geo, n_atoms, max_neighbors, view, *ctx, &need);
  for (int k = 0; k < 9; ++k) view.box.h[k] = geo.box.h[k];
  for (int k = 0; k < 9; ++k) view.box.hinv[k] = geo.box.hinv[k];
  view.skin = geo.skin;
  view.rc_list_r = geo.rc_list_r;
  view.rc_list_a = geo.rc_list_a;
  view.use_cells = geo.use_cells;
  for (int a = 0; a < 3; ++a) {
    view.nc[a] = geo.nc[a];
    view.kimg[a] = geo.kimg[a];
  }
  view.n = n_atoms;
  view.cap = max_neighbors;
  view.cells_zeroed_for = -1;  // the workspace holds the last call's contents
  ctx->sys = view;
  ctx->species_n = 0;  // one species
  ctx->have_masses = false;
  System& s = ctx->sys;
  if (n_atoms > 0) {
    launch_iota(ctx, n_atoms, s.perm.ptr);
    st = check_hip(ctx,
                   hipMemcpyAsync(s.pos_s.ptr, pos_dev, sizeof(double) * 3 * n_atoms,
                                  hipMemcpyDeviceToDevice, ctx->stream),
                   "copying positions");
    if (st != NEP_OK) return st;
    st = build_neighbors(ctx, false, false);
    if (st != NEP_OK) return st;
    launch_take_rows(ctx, n_atoms, 3, pos_dev, s.pos_s.ptr);
    if (vel_dev) launch_take_rows(ctx, n_atoms, 3, vel_dev, s.vel_s.ptr);
  }
  hipError_t e = evaluate_internal(ctx, vel_dev != nullptr,
                                   totals_dev ? totals_dev : ctx->totals.ptr, 0, 0.0, 1.0,
                                   W_dev != nullptr, J_dev != nullptr);
  if (e == hipSuccess) {
    launch_put_rows(ctx, n_atoms, 3, ctx->F.ptr, F_dev);
    if (U_dev) launch_put_rows(ctx, n_atoms, 1, ctx->U.ptr, U_dev);
    if (W_dev) launch_put_rows(ctx, n_atoms, 9, ctx->W.ptr, W_dev);
    if (J_dev) launch_put_rows(ctx, n_atoms, 3, ctx->J.ptr, J_dev);
    e = hipGetLastError();
  }
  return check_hip(ctx, e, "launching force kernels");
}

}  // extern "C"
