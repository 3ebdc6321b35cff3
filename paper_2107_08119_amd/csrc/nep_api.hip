// C ABI entry points of libnep: argument checks, state, buffer management and
// launch sequencing.  The arithmetic lives in the kernels.
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "nep_internal.h"

namespace nep {

nep_status fail(nep_ctx ctx, nep_status code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

nep_status check_hip(nep_ctx ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return NEP_OK;
  return fail(ctx, e == hipErrorOutOfMemory ? NEP_ENOMEM : NEP_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

int n_des_of(const nep_hyper& h) {
  return (h.n_max_radial + 1) + (h.n_max_angular + 1) * h.l_max;
}

namespace {

bool hyper_valid(const nep_hyper* h) {
  return h && std::isfinite(h->rc_radial) && std::isfinite(h->rc_angular) && h->rc_angular > 0 &&
         h->rc_angular <= h->rc_radial && h->n_max_radial >= 0 && h->n_max_angular >= 0 &&
         h->l_max >= 1 && h->l_max <= 4 && h->n_neuron >= 1 && h->n_max_radial < 64 &&
         h->n_max_angular < 64 && h->n_neuron <= 4096;
}

// Buffers whose size follows the system: partial forces, energies, forces,
// block partial sums.
nep_status size_system_buffers(nep_ctx ctx) {
  const System& s = ctx->sys;
  hipError_t e;
  System& sm = ctx->sys;
  if ((e = ctx->p.ensure((size_t)s.cap * s.n)) != hipSuccess ||
      (s.n <= kPairVectorMaxAtoms && (e = ctx->geo.ensure((size_t)s.cap * s.n)) != hipSuccess) ||
      (e = ctx->U.ensure((size_t)s.n)) != hipSuccess ||
      (e = ctx->fown.ensure((size_t)3 * s.n)) != hipSuccess ||
      (e = ctx->F.ensure((size_t)3 * s.n)) != hipSuccess ||
      (e = ctx->W.ensure((size_t)9 * s.n)) != hipSuccess ||
      (e = ctx->J.ensure((size_t)3 * s.n)) != hipSuccess ||
      (e = sm.pos_s.ensure((size_t)3 * s.n)) != hipSuccess ||
      (e = sm.pos_t.ensure((size_t)3 * s.n)) != hipSuccess ||
      (e = sm.vel_s.ensure((size_t)3 * s.n)) != hipSuccess ||
      (e = sm.perm.ensure((size_t)s.n)) != hipSuccess ||
      (e = ctx->partials.ensure(gather_blocks(s.n) * 16 + 16)) != hipSuccess)
    return check_hip(ctx, e, "allocating system buffers");
  return NEP_OK;
}

}  // namespace

hipError_t evaluate_internal(nep_ctx ctx, bool vel, double* out, int mode, double kick,
                             double mass, bool want_w, bool want_j, double* block_out, double dt,
                             double* pos_next, const double* fe) {
  static const double kNoField[3] = {0.0, 0.0, 0.0};
  if (!fe) fe = kNoField;
  System& s = ctx->sys;
  hipError_t e = timed(ctx, 0, [&] { return launch_partials(ctx, s.pos_s.ptr); });
  if (e != hipSuccess) return e;
  double* sums = block_out ? block_out : ctx->partials.ptr;
  return timed(ctx, 1, [&] {
    hipError_t r = launch_gather(ctx, s.pos_s.ptr, vel ? s.vel_s.ptr : nullptr, nullptr,
                                 ctx->F.ptr, want_w ? ctx->W.ptr : nullptr,
                                 want_j ? ctx->J.ptr : nullptr, sums, mode, kick, mass, dt,
                                 pos_next, fe, block_out != nullptr);
    if (r != hipSuccess || block_out) return r;
    return launch_finalize(ctx, mode == 0 ? 13 : 5, 1, sums, out, s.n == 0);
  });
}

nep_status check_box(nep_ctx ctx, const double* box_host, double skin, System& probe) {
  if (!box_host) return fail(ctx, NEP_EINVAL, "box_host is NULL");
  if (!(skin >= 0.0) || !std::isfinite(skin)) return fail(ctx, NEP_EINVAL, "skin must be >= 0");
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(box_host[k])) return fail(ctx, NEP_EINVAL, "box has non-finite entries");
  prepare_system_geometry(probe, box_host, ctx->hyper.rc_radial, ctx->hyper.rc_angular, skin);
  const double* h = probe.box.h;
  const double det = h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
                     h[2] * (h[3] * h[7] - h[4] * h[6]);
  if (!(std::fabs(det) > 0.0)) return fail(ctx, NEP_EINVAL, "box is singular");
  if (!probe.use_cells && (probe.kimg[0] > 2 || probe.kimg[1] > 2 || probe.kimg[2] > 2))
    return fail(ctx, NEP_EINVAL, "box thinner than half the list cutoff along a cell vector");
  return NEP_OK;
}

}  // namespace nep

using namespace nep;

extern "C" {

nep_status nep_create(nep_ctx* out, int device, void* hip_stream) {
  if (!out) return NEP_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return NEP_EINVAL;
  DeviceGuard guard(device);
  nep_ctx ctx = new (std::nothrow) nep_ctx_s();
  if (!ctx) return NEP_ENOMEM;
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  hipError_t e;
  if ((e = ctx->flags.ensure(kNumFlags)) != hipSuccess || (e = ctx->totals.ensure(16)) != hipSuccess ||
      (e = hipMemset(ctx->flags.ptr, 0, sizeof(int) * kNumFlags)) != hipSuccess) {
    nep_destroy(ctx);
    return e == hipErrorOutOfMemory ? NEP_ENOMEM : NEP_EDEVICE;
  }
  scratch_setup(device);
  *out = ctx;
  return NEP_OK;
}

void nep_destroy(nep_ctx ctx) {
  if (!ctx) return;
  DeviceGuard guard(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->sys.release();
  ctx->z.release();
  ctx->p.release();
  ctx->geo.release();
  ctx->species_w.release();
  ctx->species_wd.release();
  ctx->masses.release();
  ctx->fown.release();
  ctx->U.release();
  ctx->F.release();
  ctx->W.release();
  ctx->J.release();
  ctx->partials.release();
  ctx->totals.release();
  ctx->flags.release();
  ctx->snes_graph.release();
  ctx->gen_counter.release();
  delete ctx;
}

const char* nep_last_error(nep_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

nep_status nep_set_stream(nep_ctx ctx, void* hip_stream) {
  if (!ctx) return NEP_EINVAL;
  ctx->stream = (hipStream_t)hip_stream;
  return NEP_OK;
}

nep_status nep_synchronize(nep_ctx ctx) {
  if (!ctx) return NEP_EINVAL;
  DeviceGuard guard(ctx->device);
  nep_status st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "synchronizing");
  if (st != NEP_OK) return st;
  int h[kNumFlags];
  st = check_hip(ctx, hipMemcpy(h, ctx->flags.ptr, sizeof(h), hipMemcpyDeviceToHost),
                 "reading device flags");
  if (st != NEP_OK) return st;
  int any = 0;
  for (int k = 0; k < kNumFlags; ++k) any |= h[k];
  if (any) {
    st = check_hip(ctx, hipMemset(ctx->flags.ptr, 0, sizeof(h)), "clearing device flags");
    if (st != NEP_OK) return st;
  }
  if (h[kFlagOverflow]) return fail(ctx, NEP_EOVERFLOW, "an atom has more than max_neighbors neighbours");
  if (h[kFlagImage]) return fail(ctx, NEP_EIMAGE, "a neighbour needs a lattice image beyond +-3 cells");
  if (h[kFlagReverse]) return fail(ctx, NEP_EDEVICE, "neighbour list is not symmetric");
  if (h[kFlagNonFinite]) return fail(ctx, NEP_ENONFINITE, "non-finite energy, virial or heat current");
  if (h[kFlagSkin])
    return fail(ctx, NEP_ESKIN,
                "an atom moved more than skin/2 since its neighbour list was built (rebuild "
                "more often or use a larger skin)");
  return NEP_OK;
}

int nep_num_descriptors(const nep_hyper* hyper) {
  return hyper_valid(hyper) ? n_des_of(*hyper) : 0;
}

int nep_num_params(const nep_hyper* hyper) {
  return hyper_valid(hyper) ? (n_des_of(*hyper) + 2) * hyper->n_neuron + 1 : 0;
}

nep_status nep_load_params(nep_ctx ctx, const nep_hyper* hyper, const float* z_host, int n_par) {
  if (!ctx) return NEP_EINVAL;
  if (!hyper_valid(hyper)) return fail(ctx, NEP_EINVAL, "invalid hyperparameters");
  if (!z_host) return fail(ctx, NEP_EINVAL, "z_host is NULL");
  const int want = nep_num_params(hyper);
  if (n_par != want)
    return fail(ctx, NEP_EINVAL,
                "n_par is " + std::to_string(n_par) + ", expected (N_des+2)*N_neu+1 = " +
                    std::to_string(want));
  if (!have_force_variant(*hyper))
    return fail(ctx, NEP_ENOTIMPL, "no compiled kernel for these descriptor/network sizes");
  if (ctx->have_list && (hyper->rc_radial != ctx->hyper.rc_radial ||
                         hyper->rc_angular != ctx->hyper.rc_angular))
    ctx->have_list = false;  // list cutoffs change with the model
  DeviceGuard guard(ctx->device);
  nep_status st = check_hip(ctx, ctx->z.ensure(n_par), "allocating parameters");
  if (st != NEP_OK) return st;
  st = check_hip(ctx,
                 hipMemcpyAsync(ctx->z.ptr, z_host, sizeof(float) * n_par, hipMemcpyHostToDevice,
                                ctx->stream),
                 "copying parameters");
  if (st != NEP_OK) return st;
  st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "copying parameters");
  if (st != NEP_OK) return st;
  ctx->hyper = *hyper;
  ctx->n_des = n_des_of(*hyper);
  ctx->n_par = n_par;
  ctx->have_params = true;
  ctx->md_forces_valid = false;
  return NEP_OK;
}

nep_status nep_build_neighbors(nep_ctx ctx, int n_atoms, const double* pos_dev,
                               const double* box_host, double skin, int max_neighbors) {
  if (!ctx) return NEP_EINVAL;
  if (!ctx->have_params) return fail(ctx, NEP_ESTATE, "nep_load_params must come first");
  if (n_atoms < 0 || n_atoms > kMaxAtoms)
    return fail(ctx, NEP_EINVAL, "n_atoms must be in [0, 2^23)");
  if (n_atoms > 0 && !pos_dev) return fail(ctx, NEP_EINVAL, "pos_dev is NULL");
  if (max_neighbors < 1 || (size_t)max_neighbors * (size_t)(n_atoms > 0 ? n_atoms : 1) >= (1ull << 31))
    return fail(ctx, NEP_EINVAL, "need 1 <= max_neighbors and max_neighbors * n_atoms < 2^31");
  System& s = ctx->sys;
  System probe;
  nep_status chk = check_box(ctx, box_host, skin, probe);
  if (chk != NEP_OK) return chk;
  DeviceGuard guard(ctx->device);
  for (int k = 0; k < 9; ++k) s.box.h[k] = probe.box.h[k];
  for (int k = 0; k < 9; ++k) s.box.hinv[k] = probe.box.hinv[k];
  s.skin = probe.skin;
  s.rc_list_r = probe.rc_list_r;
  s.rc_list_a = probe.rc_list_a;
  s.use_cells = probe.use_cells;
  for (int a = 0; a < 3; ++a) {
    s.nc[a] = probe.nc[a];
    s.kimg[a] = probe.kimg[a];
  }
  if (ctx->species_n != n_atoms) {  // species describe another system
    ctx->species_n = 0;
    ctx->have_masses = false;
  }
  s.n = n_atoms;
  s.cap = max_neighbors;
  ctx->have_list = false;
  ctx->md_forces_valid = false;
  nep_status st = size_system_buffers(ctx);
  if (st != NEP_OK) return st;
  if (n_atoms > 0) {
    launch_iota(ctx, n_atoms, s.perm.ptr);
    st = check_hip(ctx,
                   hipMemcpyAsync(s.pos_s.ptr, pos_dev, sizeof(double) * 3 * n_atoms,
                                  hipMemcpyDeviceToDevice, ctx->stream),
                   "copying positions");
    if (st != NEP_OK) return st;
    st = build_neighbors(ctx, false, false);
    if (st != NEP_OK) return st;
  }
  ctx->have_list = true;
  ctx->steps_since_rebuild = 0;
  return NEP_OK;
}

nep_status nep_set_species(nep_ctx ctx, int n, const int* atomic_numbers_host,
                           const double* masses_amu_host) {
  if (!ctx) return NEP_EINVAL;
  if (!atomic_numbers_host) {
    ctx->species_n = 0;
    ctx->have_masses = false;
    ctx->md_forces_valid = false;
    return NEP_OK;
  }
  if (!ctx->have_list) return fail(ctx, NEP_ESTATE, "nep_build_neighbors must come first");
  if (n != ctx->sys.n || n < 1) return fail(ctx, NEP_EINVAL, "n must equal the system's atom count");
  std::vector<float> w((size_t)n);
  std::vector<double> wd((size_t)n);
  for (int k = 0; k < n; ++k) {
    const int Z = atomic_numbers_host[k];
    if (Z < 1 || Z > 118) return fail(ctx, NEP_EINVAL, "atomic numbers must be in 1..118");
    wd[k] = std::sqrt((double)Z);
    w[k] = (float)wd[k];
  }
  if (masses_amu_host)
    for (int k = 0; k < n; ++k)
      if (!(masses_amu_host[k] > 0.0) || !std::isfinite(masses_amu_host[k]))
        return fail(ctx, NEP_EINVAL, "masses must be > 0");
  DeviceGuard guard(ctx->device);
  hipError_t e = ctx->species_w.ensure((size_t)n);
  if (e == hipSuccess) e = ctx->species_wd.ensure((size_t)n);
  if (e == hipSuccess && masses_amu_host) e = ctx->masses.ensure((size_t)n);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpy(ctx->species_w.ptr, w.data(), sizeof(float) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(ctx->species_wd.ptr, wd.data(), sizeof(double) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess && masses_amu_host)
    e = hipMemcpy(ctx->masses.ptr, masses_amu_host, sizeof(double) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    ctx->species_n = 0;
    ctx->have_masses = false;
    return check_hip(ctx, e, "copying species");
  }
  ctx->species_n = n;
  ctx->have_masses = masses_amu_host != nullptr;
  ctx->md_forces_valid = false;
  return NEP_OK;
}

nep_status nep_get_neighbors(nep_ctx ctx, int* cnt_radial_dev, int* cnt_angular_dev, int* nbr_dev,
                             int* img_dev, int* rev_dev) {
  if (!ctx) return NEP_EINVAL;
  if (!ctx->have_list) return fail(ctx, NEP_ESTATE, "no neighbour list");
  if (ctx->sys.n == 0) return NEP_OK;
  DeviceGuard guard(ctx->device);
  return check_hip(ctx,
                   unpack_neighbors(ctx, nbr_dev, img_dev, cnt_radial_dev, cnt_angular_dev, rev_dev),
                   "unpacking neighbour list");
}

nep_status nep_compute(nep_ctx ctx, const double* pos_dev, const double* vel_dev, float* U_dev,
                       float* F_dev, float* W_dev, float* J_dev, double* totals_dev) {
  if (!ctx) return NEP_EINVAL;
  if (!ctx->have_params || !ctx->have_list)
    return fail(ctx, NEP_ESTATE, "nep_load_params and nep_build_neighbors must come first");
  System& s = ctx->sys;
  const int n = s.n;
  if (n > 0 && (!pos_dev || !F_dev)) return fail(ctx, NEP_EINVAL, "pos_dev and F_dev are required");
  if (J_dev && !vel_dev) return fail(ctx, NEP_EINVAL, "J_dev needs vel_dev");
  DeviceGuard guard(ctx->device);
  ctx->md_forces_valid = false;
  launch_take_rows(ctx, n, 3, pos_dev, s.pos_s.ptr);
  if (vel_dev) launch_take_rows(ctx, n, 3, vel_dev, s.vel_s.ptr);
  hipError_t e = evaluate_internal(ctx, vel_dev != nullptr,
                                   totals_dev ? totals_dev : ctx->totals.ptr, 0, 0.0, 1.0,
                                   W_dev != nullptr, J_dev != nullptr);
  if (e == hipSuccess) {
    launch_put_rows(ctx, n, 3, ctx->F.ptr, F_dev);
    if (U_dev) launch_put_rows(ctx, n, 1, ctx->U.ptr, U_dev);
    if (W_dev) launch_put_rows(ctx, n, 9, ctx->W.ptr, W_dev);
    if (J_dev) launch_put_rows(ctx, n, 3, ctx->J.ptr, J_dev);
    e = hipGetLastError();
  }
  return check_hip(ctx, e, "launching force kernels");
}

nep_status nep_md_step(nep_ctx ctx, int n_steps, double dt_fs, int rebuild_every,
                       double mass_amu, double* pos_dev, double* vel_dev, double* thermo_dev,
                       float* W_dev, float* J_dev) {
  const double none[3] = {0.0, 0.0, 0.0};
  return nep_md_step_driven(ctx, n_steps, dt_fs, rebuild_every, mass_amu, none, pos_dev,
                            vel_dev, thermo_dev, W_dev, J_dev);
}

nep_status nep_md_step_driven(nep_ctx ctx, int n_steps, double dt_fs, int rebuild_every,
                              double mass_amu, const double* fe_host, double* pos_dev,
                              double* vel_dev, double* thermo_dev, float* W_dev, float* J_dev) {
  if (!ctx) return NEP_EINVAL;
  if (!ctx->have_params || !ctx->have_list)
    return fail(ctx, NEP_ESTATE, "nep_load_params and nep_build_neighbors must come first");
  if (n_steps < 0) return fail(ctx, NEP_EINVAL, "n_steps must be >= 0");
  if (!(dt_fs > 0.0) || !std::isfinite(dt_fs)) return fail(ctx, NEP_EINVAL, "dt must be > 0");
  if (rebuild_every < 1) return fail(ctx, NEP_EINVAL, "rebuild_every must be >= 1");
  if (!(mass_amu > 0.0) || !std::isfinite(mass_amu)) return fail(ctx, NEP_EINVAL, "mass must be > 0");
  if (!fe_host) return fail(ctx, NEP_EINVAL, "fe_host is NULL");
  for (int c = 0; c < 3; ++c)
    if (!std::isfinite(fe_host[c])) return fail(ctx, NEP_EINVAL, "fe has non-finite entries");
  if (n_steps == 0) return NEP_OK;
  System& s = ctx->sys;
  const int n = s.n;
  if (n > 0 && (!pos_dev || !vel_dev)) return fail(ctx, NEP_EINVAL, "pos/vel are required");
  if (!thermo_dev) return fail(ctx, NEP_EINVAL, "thermo_dev is required");
  DeviceGuard guard(ctx->device);
  const double kick = 0.5 * dt_fs * kAccel / mass_amu;
  // Thermo block sums of up to `chunk` steps are kept and reduced together.
  const size_t nb = gather_blocks(n);
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(64, ((size_t)4 << 20) / (nb * 5 + 1)));
  hipError_t e = ctx->partials.ensure((size_t)chunk * nb * 5 + 16);
  if (e != hipSuccess) return check_hip(ctx, e, "allocating thermo sums");
  const bool same_field = ctx->md_fe[0] == fe_host[0] && ctx->md_fe[1] == fe_host[1] &&
                          ctx->md_fe[2] == fe_host[2];
  const bool forces_valid =
      ctx->md_forces_valid && ctx->md_pos == pos_dev && ctx->md_vel == vel_dev && same_field;
  ctx->md_forces_valid = false;
  int pending = 0;
  // The caller's arrays in the internal (cell) order and the first half-kick
  // and drift of step 0 (later steps get theirs from the previous step's
  // pass 2): one kernel when the kept forces belong to these positions,
  // else the forces of the starting positions first (with the driving force:
  // mode 1 with a zero kick computes F + F_e . W and leaves the velocities
  // unchanged).
  if (forces_valid) {
    e = timed(ctx, 3, [&] {
      return launch_take_kick_drift(ctx, pos_dev, vel_dev, s.pos_s.ptr, s.vel_s.ptr, kick,
                                    mass_amu, dt_fs);
    });
    if (e != hipSuccess) return check_hip(ctx, e, "launching integrator");
  } else {
    launch_take_rows(ctx, n, 3, pos_dev, s.pos_s.ptr);
    launch_take_rows(ctx, n, 3, vel_dev, s.vel_s.ptr);
    e = evaluate_internal(ctx, true, nullptr, 1, 0.0, mass_amu, false, false, ctx->partials.ptr,
                          0.0, nullptr, fe_host);
    if (e != hipSuccess) return check_hip(ctx, e, "launching force kernels");
    e = timed(ctx, 3, [&] {
      return launch_kick_drift(ctx, s.pos_s.ptr, s.vel_s.ptr, kick, mass_amu, dt_fs);
    });
    if (e != hipSuccess) return check_hip(ctx, e, "launching integrator");
  }
  for (int step = 0; step < n_steps; ++step) {
    if (++ctx->steps_since_rebuild >= rebuild_every) {
      if (n > 0) {
        nep_status st = NEP_OK;
        e = timed(ctx, 2, [&] {
          st = build_neighbors(ctx, true, true);
          return st == NEP_OK ? hipSuccess : hipErrorUnknown;
        });
        if (st != NEP_OK) return st;
        if (e != hipSuccess) return check_hip(ctx, e, "timing neighbour build");
      }
      ctx->steps_since_rebuild = 0;
    }
    const bool last = step == n_steps - 1;
    e = evaluate_internal(ctx, true, nullptr, last ? 1 : 2, kick, mass_amu, W_dev != nullptr,
                          J_dev != nullptr,
                          ctx->partials.ptr + (size_t)pending * nb * 5, dt_fs,
                          last ? nullptr : s.pos_t.ptr, fe_host);
    if (e != hipSuccess) return check_hip(ctx, e, "launching force kernels");
    if (!last && n > 0) s.pos_s.swap(s.pos_t);
    // per-atom W and J of this step in the caller's order (the gather writes
    // them in cell order: coalesced, then one scatter pass each)
    if (W_dev) launch_put_rows(ctx, n, 9, ctx->W.ptr, W_dev);
    if (J_dev) launch_put_rows(ctx, n, 3, ctx->J.ptr, J_dev);
    if (++pending == chunk || last) {
      e = timed(ctx, 3, [&] {
        return launch_finalize(ctx, 5, pending, ctx->partials.ptr,
                               thermo_dev + (size_t)5 * (step + 1 - pending), true);
      });
      if (e != hipSuccess) return check_hip(ctx, e, "launching thermo sums");
      pending = 0;
    }
  }
  launch_put_rows2(ctx, n, s.pos_s.ptr, pos_dev, s.vel_s.ptr, vel_dev);
  e = hipGetLastError();
  if (e != hipSuccess) return check_hip(ctx, e, "copying the state back");
  ctx->md_forces_valid = true;
  ctx->md_pos = pos_dev;
  ctx->md_vel = vel_dev;
  for (int c = 0; c < 3; ++c) ctx->md_fe[c] = fe_host[c];
  return NEP_OK;
}

nep_status nep_set_timing(nep_ctx ctx, int enable) {
  if (!ctx) return NEP_EINVAL;
  ctx->timer.on = enable != 0;
  for (int c = 0; c < KernelTimer::kClasses; ++c) ctx->timer.used[c] = 0;
  return NEP_OK;
}

nep_status nep_get_timing(nep_ctx ctx, double* ms_out, int* launches_out) {
  if (!ctx || !ms_out || !launches_out) return NEP_EINVAL;
  DeviceGuard guard(ctx->device);
  nep_status st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "synchronizing");
  if (st != NEP_OK) return st;
  KernelTimer& t = ctx->timer;
  for (int c = 0; c < KernelTimer::kClasses; ++c) {
    double tot = 0.0;
    for (size_t k = 0; k < t.used[c]; ++k) {
      float ms = 0.f;
      st = check_hip(ctx, hipEventElapsedTime(&ms, t.start[c][k], t.stop[c][k]), "reading events");
      if (st != NEP_OK) return st;
      tot += ms;
    }
    ms_out[c] = tot;
    launches_out[c] = (int)t.used[c];
    t.used[c] = 0;
  }
  return NEP_OK;
}

nep_status nep_time_partials(nep_ctx ctx, const double* pos_dev, int reps, double* ms_per_launch) {
  if (!ctx || !ms_per_launch) return NEP_EINVAL;
  if (!ctx->have_params || !ctx->have_list)
    return fail(ctx, NEP_ESTATE, "nep_load_params and nep_build_neighbors must come first");
  if (reps < 1 || reps > 100000) return fail(ctx, NEP_EINVAL, "reps must be in [1, 100000]");
  if (ctx->sys.n > 0 && !pos_dev) return fail(ctx, NEP_EINVAL, "pos_dev is NULL");
  DeviceGuard guard(ctx->device);
  launch_take_rows(ctx, ctx->sys.n, 3, pos_dev, ctx->sys.pos_s.ptr);
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipEventRecord(a, ctx->stream);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_partials(ctx, ctx->sys.pos_s.ptr);
  if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e != hipSuccess) return check_hip(ctx, e, "timing the partial-force kernel");
  *ms_per_launch = (double)ms / reps;
  ctx->md_forces_valid = false;  // the partial forces were recomputed
  return NEP_OK;
}

nep_status nep_autotune(nep_ctx ctx, const double* pos_dev, int reps, int* lanes_out,
                        double* ms_out) {
  if (!ctx) return NEP_EINVAL;
  if (!ctx->have_params || !ctx->have_list)
    return fail(ctx, NEP_ESTATE, "nep_load_params and nep_build_neighbors must come first");
  if (reps < 1 || reps > 10000) return fail(ctx, NEP_EINVAL, "reps must be in [1, 10000]");
  if (ctx->sys.n > 0 && !pos_dev) return fail(ctx, NEP_EINVAL, "pos_dev is NULL");
  DeviceGuard guard(ctx->device);
  launch_take_rows(ctx, ctx->sys.n, 3, pos_dev, ctx->sys.pos_s.ptr);
  const bool timing = ctx->timer.on;
  ctx->timer.on = false;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  int best = ctx->md_variant;
  // other model sizes have the one-wave-per-atom kernel only
  const int nv = have_training_variant(ctx->hyper) && !ctx->species_on() ? 3 : 1;
  // shapes timed in interleaved rounds; each keeps its fastest round
  constexpr int kRounds = 3;
  double per[3] = {0.0, 0.0, 0.0};
  for (int round = 0; round < kRounds && e == hipSuccess; ++round)
    for (int v = 0; v < nv && e == hipSuccess; ++v) {
      if (round == 0) e = launch_partials(ctx, ctx->sys.pos_s.ptr, v);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(a, ctx->stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r)
        e = launch_partials(ctx, ctx->sys.pos_s.ptr, v);
      if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e == hipSuccess && (round == 0 || (double)ms / reps < per[v])) per[v] = (double)ms / reps;
    }
  if (e == hipSuccess) {
    best = 0;
    for (int v = 1; v < nv; ++v)
      if (per[v] < per[best]) best = v;
  }
  if (ms_out)
    for (int v = 0; v < 3; ++v) ms_out[v] = per[v < nv ? v : 0];
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  ctx->timer.on = timing;
  ctx->md_forces_valid = false;  // the partial forces were recomputed
  if (e != hipSuccess) return check_hip(ctx, e, "timing the partial-force kernel");
  ctx->md_variant = nv == 3 ? best : 3;
  if (lanes_out) *lanes_out = nv == 3 ? 2 << best : 64;
  return NEP_OK;
}

nep_status nep_set_tile(nep_ctx ctx, int lanes) {
  if (!ctx) return NEP_EINVAL;
  if (lanes != 2 && lanes != 4 && lanes != 8 && lanes != 64)
    return fail(ctx, NEP_EINVAL, "lanes must be 2, 4, 8 or 64");
  ctx->md_variant = lanes == 2 ? 0 : (lanes == 4 ? 1 : (lanes == 8 ? 2 : 3));
  ctx->md_forces_valid = false;
  return NEP_OK;
}

}  // extern "C"
