// Internal declarations of libnep (gfx950).  Not part of the C ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "nep.h"

namespace nep {

// A periodic cell: rows of h are the cell vectors; hinv is its inverse, so
// fractional coordinates are s = r . hinv (row vector times matrix).
struct Box {
  double h[9];
  double hinv[9];
};

// Packed neighbour entry: atom index in the low 23 bits, lattice image
// n0+3, n1+3, n2+3 (each 0..6) in three 3-bit fields of the high 9 bits.
constexpr int kAtomBits = 23;
constexpr uint32_t kAtomMask = (1u << kAtomBits) - 1u;
constexpr int kMaxAtoms = (1 << kAtomBits) - 1;

__host__ __device__ inline uint32_t pack_entry(int j, int n0, int n1, int n2) {
  return (uint32_t)j | ((uint32_t)((n0 + 3) | ((n1 + 3) << 3) | ((n2 + 3) << 6)) << kAtomBits);
}
__host__ __device__ inline void unpack_image(uint32_t e, int& n0, int& n1, int& n2) {
  n0 = (int)((e >> kAtomBits) & 7u) - 3;
  n1 = (int)((e >> (kAtomBits + 3)) & 7u) - 3;
  n2 = (int)(e >> (kAtomBits + 6)) - 3;
}

// Pass 1 hands pass 2 the pair vectors r_ij (12 bytes per list slot) for
// systems of up to 2^17 atoms, whose vectors stay in the chip's last-level
// cache between the two passes; for larger systems writing them to HBM costs
// pass 1 more than it saves pass 2, which then forms r_ij again from the
// list and the positions.
constexpr int kPairVectorMaxAtoms = 1 << 17;

// A device array owned by the context that only grows, or (view) a fixed
// range of memory owned elsewhere, which it never frees or grows.
template <class T>
struct DevBuf {
  T* ptr = nullptr;
  size_t size = 0;
  bool view = false;
  void set_view(T* p, size_t n) {
    ptr = p;
    size = n;
    view = true;
  }
  hipError_t ensure(size_t need) {
    if (ptr && need <= size) return hipSuccess;
    if (view) return hipErrorOutOfMemory;
    if (ptr) {
      hipError_t e = hipFree(ptr);
      ptr = nullptr;
      size = 0;
      if (e != hipSuccess) return e;
    }
    size_t n = need > 0 ? need : 1;
    hipError_t e = hipMalloc((void**)&ptr, n * sizeof(T));
    if (e != hipSuccess) {
      ptr = nullptr;
      return e;
    }
    size = n;
    return hipSuccess;
  }
  void release() {
    if (ptr && !view) (void)hipFree(ptr);
    ptr = nullptr;
    size = 0;
    view = false;
  }
  void swap(DevBuf& o) {
    T* p = ptr;
    ptr = o.ptr;
    o.ptr = p;
    size_t z = size;
    size = o.size;
    o.size = z;
    bool v = view;
    view = o.view;
    o.view = v;
  }
};

// Device error flags latched by kernels.
enum Flag {
  kFlagOverflow = 0,
  kFlagImage = 1,
  kFlagNonFinite = 2,
  kFlagReverse = 3,
  kFlagSkin = 4,  // an evaluation saw an atom more than skin/2 from its list-build position
  kNumFlags = 5
};

// 1 eV/A acting on 1 amu, in A/fs^2; and 1 amu A^2/fs^2 in eV.
constexpr double kAccel = 1.602176634e-19 / 1.66053906660e-27 * 1.0e-10;

// An atom as a neighbour candidate, stored in cell order: float64 position,
// index, and integer cell offsets of the raw position packed as 3 x int8.
// One stored partial force dU_i/dr_ij: 12 bytes (one dwordx3 access).
struct Partial3 {
  float x, y, z;
};

struct alignas(32) CellRec {
  double x, y, z;
  int j;
  int w;
};

// Neighbour-list state of one system (a single periodic box).
struct System {
  int n = 0;             // atoms
  int cap = 0;           // slots per atom (max_neighbors)
  Box box{};
  double skin = 0.0;
  double rc_list_r = 0, rc_list_a = 0;  // rc + skin
  bool use_cells = false;
  int cells_zeroed_for = -1;  // cell_cnt is known zero for this cell count (-1: unknown)
  int nc[3] = {1, 1, 1};
  int kimg[3] = {0, 0, 0};  // image range for the all-pairs builder
  // device arrays (owned by the context)
  DevBuf<uint32_t> nl;     // [cap][n]
  DevBuf<uint32_t> nl_rm;  // [n][cap] the same entries per atom (reverse-slot search)
  DevBuf<int> cnt_r;       // [n]
  DevBuf<int> cnt_a;       // [n]
  DevBuf<int> rev;         // [cap][n]
  DevBuf<int> wrap;        // [3][n] integer cell offsets of the raw positions
  DevBuf<int> cell_of;     // [n]
  DevBuf<int> cell_cnt;    // [ncell]
  DevBuf<int> cell_start;  // [ncell+1]
  DevBuf<int> cell_fill;   // [ncell]
  DevBuf<int> scan_part;   // [1024] block totals of the multi-block cell scan
  DevBuf<int> cell_atoms;  // [n] members of each cell, in arrival order
  DevBuf<CellRec> cell_rec;  // [n] positions and offsets in cell order
  DevBuf<float> pos_ref;     // [3][n] positions at the last list build (float32, internal order)
  // The library works on its own copies of positions and velocities in cell
  // order (re-sorted at every rebuild); perm[k] is the caller's index of the
  // atom at internal index k, iperm[c] the internal index of caller atom c.
  DevBuf<double> pos_s, pos_t;  // [3][n]
  DevBuf<double> vel_s, vel_t;  // [3][n]
  DevBuf<int> perm, perm_t;     // [n]
  DevBuf<int> iperm;            // [n]
  DevBuf<int> wrap_t, cell_t;   // [3][n], [n]
  void release() {
    nl.release();
    nl_rm.release();
    cnt_r.release();
    cnt_a.release();
    rev.release();
    wrap.release();
    cell_of.release();
    cell_cnt.release();
    cell_start.release();
    cell_fill.release();
    scan_part.release();
    cell_atoms.release();
    cell_rec.release();
    pos_s.release();
    pos_t.release();
    vel_s.release();
    vel_t.release();
    perm.release();
    perm_t.release();
    iperm.release();
    wrap_t.release();
    cell_t.release();
  }
};

// Event pairs bracketing kernel launches, per kernel class.
struct KernelTimer {
  static constexpr int kClasses = 4;
  bool on = false;
  std::vector<hipEvent_t> start[kClasses], stop[kClasses];
  size_t used[kClasses] = {0, 0, 0, 0};
  ~KernelTimer() {
    for (int c = 0; c < kClasses; ++c) {
      for (hipEvent_t e : start[c]) (void)hipEventDestroy(e);
      for (hipEvent_t e : stop[c]) (void)hipEventDestroy(e);
    }
  }
};

}  // namespace nep

namespace nep {
// A generation of snes_run captured as a HIP graph, with everything it was
// captured for (pointers, sizes, rates, kernel shape).
struct SnesGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> ptr_key;
  std::vector<double> val_key;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    ptr_key.clear();
    val_key.clear();
  }
};
}  // namespace nep

struct nep_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  // model
  bool have_params = false;
  nep_hyper hyper{};
  int n_des = 0, n_par = 0;
  nep::DevBuf<float> z;  // [n_par]
  // system
  bool have_list = false;
  nep::System sys;
  nep::DevBuf<nep::Partial3> p;   // incoming partial forces dU_j/dr_ji at i's slots, [cap][n]
  nep::DevBuf<nep::Partial3> geo; // pair vectors r_ij of i's slots from pass 1, [cap][n]
  nep::DevBuf<float> fown;        // sum_j dU_i/dr_ij, [3][n]
  nep::DevBuf<float> U;           // [n]
  nep::DevBuf<float> F;           // [3][n]
  nep::DevBuf<float> W;           // [9][n] internal per-atom virials
  nep::DevBuf<float> J;           // [3][n] internal heat currents
  nep::DevBuf<double> partials;   // [blocks][16] block sums
  int md_variant = 1;             // pass-1 tile shape: 0, 1, 2, 3 = 2, 4, 8, 64 lanes per atom
  // multicomponent system (caller order): sqrt(Z) per atom and optional masses
  int species_n = 0;              // atoms the arrays describe; 0 = one species
  bool have_masses = false;
  nep::DevBuf<float> species_w;   // [n] sqrt(atomic number)
  nep::DevBuf<double> species_wd;  // [n] the same in float64 (descriptor sums)
  nep::DevBuf<double> masses;     // [n] amu
  nep::DevBuf<double> totals;     // [16]
  nep::DevBuf<int> flags;         // [kNumFlags]
  // molecular dynamics state
  bool md_forces_valid = false;
  const double* md_pos = nullptr;
  const double* md_vel = nullptr;
  double md_fe[3] = {0.0, 0.0, 0.0};  // driving force included in the kept forces
  int steps_since_rebuild = 0;
  nep::KernelTimer timer;
  // events of the kernel class being launched (set by nep::timed)
  hipEvent_t ev_first = nullptr, ev_last = nullptr;
  // snes_run: generation counter and first generation of the call, and the
  // captured generation
  nep::DevBuf<int> gen_counter;  // [2]
  nep::SnesGraph snes_graph;
  // species weights and masses apply to the current system
  bool species_on() const { return species_n > 0 && species_n == sys.n; }
};

// A training set on the device (structures concatenated).
struct nep_dataset_s {
  nep_ctx ctx = nullptr;
  int S = 0, N = 0, cap = 0;
  int n_virial = 0;
  double rc_r = 0, rc_a = 0;  // cutoffs the lists were built for
  nep::DevBuf<double> pos;     // [3][N] wrapped
  nep::DevBuf<double> boxes;   // [S][9]
  nep::DevBuf<double> boxinv;  // [S][9]
  nep::DevBuf<int> struct_of;  // [N]
  nep::DevBuf<int> off;        // [S+1]
  nep::DevBuf<int> kimg;       // [S][3]
  nep::DevBuf<double> e_tar;   // [S]
  nep::DevBuf<double> f_tar;   // [3][N]
  nep::DevBuf<double> w_tar;   // [S][6]
  nep::DevBuf<int> has_v;      // [S]
  nep::DevBuf<uint32_t> nl;    // [cap][N]
  nep::DevBuf<int> cnt_r, cnt_a, rev, wrap;
  // geometry cache for population evaluation (positions are fixed)
  nep::DevBuf<float4> prec;    // [cap][N] compacted in-range pairs: r_ij, reverse record
  nep::DevBuf<int> pcidx;      // [cap][N] compacted index of each list slot, or -1
  nep::DevBuf<int> pn_ang;     // [N] pairs inside r_c^A (they come first)
  nep::DevBuf<int> pn_in;      // [N] pairs inside a cutoff
  nep::DevBuf<float> desc;     // [N][152] q_i (29) and c_nlm (120), padded
  std::vector<int> off_host;   // [S+1] first atom of each structure
  // Population operands (geometry only, rebuilt with the positions): the
  // padded descriptors, and per atom the derivatives of its descriptor with
  // respect to its pair vectors in matrix-core fragment order (see
  // population.hip); structures grouped into tiles of at most tile_max atoms.
  nep::DevBuf<float> qpad;       // [N][32]
  nep::DevBuf<float> pfrag;      // [chunks][64]
  nep::DevBuf<float4> ppair;     // [sum of pairs] unit vector and receiver index in its tile
  nep::DevBuf<int4> pmeta;       // [N] first chunk, first pair, pairs, angular pairs
  nep::DevBuf<int> tile_off;     // [T+1] first atom of each tile
  nep::DevBuf<int> tile_s0;      // [T+1] first structure of each tile
  nep::DevBuf<int> tile_order;   // [T] tiles by decreasing work
  nep::DevBuf<int> stile0;       // [S] first atom of the tile holding structure s
  nep::DevBuf<float2> pnorm;     // [N] largest row 1-norm of the force rows, of the virial rows
  nep::DevBuf<float2> tbound;    // [T] fixed-point bound factors of forces and virials
  int n_tiles = 0, tile_max = 0;
  long long pairs_r = 0, pairs_a = 0;  // pairs inside r_c^R, inside r_c^A (geometry cache)
  int tile_kc = 0;               // individuals per contraction launch the tiles were sized for
  int pop_variant = 1;         // network kernel shape: 0, 1, 2 = 16, 32, 64 atoms per wave
  unsigned long long serial = 0;  // unique per dataset created by the process
  bool pop_tuned = false;
  // population workspace
  nep::DevBuf<nep::Partial3> pin;   // [cap][N] partial forces (nep_dataset_compute)
  nep::DevBuf<float> fown;          // [3][N]
  nep::DevBuf<float> U;             // [pop][N]
  nep::DevBuf<float> dq;            // [pop][N][32] dU/dq of every individual
  nep::DevBuf<float> dqbound;       // [pop] bound on |dU/dq| of every individual
  nep::DevBuf<float4> wfrag;        // [pop][12][64] network weights in fragment order
  nep::DevBuf<float> wb2;           // [pop] output biases
  nep::DevBuf<double> atom_terms;   // [10][N] per-atom U and W (forward)
  nep::DevBuf<double> struct_sq;    // [pop][S][3] squared errors per structure
  // backward workspace
  nep::DevBuf<float> grad_rec;      // [fields][N]
  nep::DevBuf<double> grad_part;    // [blocks][N_par]
  void release_cache() {
    prec.release();
    pcidx.release();
    pn_ang.release();
    pn_in.release();
    desc.release();
    qpad.release();
    pfrag.release();
    ppair.release();
    pmeta.release();
    tile_off.release();
    tile_s0.release();
    tile_order.release();
    stile0.release();
    pnorm.release();
    tbound.release();
  }
};

namespace nep {

// population.hip
// Pair records and per-atom descriptors of a dataset's current positions.
hipError_t prepare_dataset_geometry(nep_ctx ctx, nep_dataset ds);
// Loss sums sq[k][s][3] of n_pop individuals (Z [n_pop][N_par]) with the
// given network-kernel shape (0..population_variants()-1).
hipError_t launch_population(nep_ctx ctx, nep_dataset ds, int n_pop, const float* Z, int variant,
                             bool first);
int population_variants();
int population_atoms(int variant);
// Largest structure snes_eval_population handles (its forces for one
// individual must fit the contraction kernel's LDS).
int population_max_structure();

// neighbours.hip
// Build the list of the internal positions sys.pos_s; on the cell path the
// atoms (positions, velocities when have_vel, perm) are first re-sorted into
// cell order.  wrap_in_place maps the internal positions into the box.
nep_status build_neighbors(nep_ctx ctx, bool wrap_in_place, bool have_vel);
// dst[r*n + k] = src[r*n + perm[k]] (caller order -> internal order).
void launch_take_rows(nep_ctx ctx, int n, int rows, const double* src, double* dst);
// dst[r*n + c] = src[r*n + iperm[c]] (internal order -> caller order; the
// same as dst[r*n + perm[k]] = src[r*n + k], with coalesced stores).
void launch_put_rows(nep_ctx ctx, int n, int rows, const double* src, double* dst);
void launch_put_rows(nep_ctx ctx, int n, int rows, const float* src, float* dst);
// both [3][n] arrays a (to a_dst) and b (to b_dst) in one launch
void launch_put_rows2(nep_ctx ctx, int n, const double* a, double* a_dst, const double* b,
                      double* b_dst);
void launch_iota(nep_ctx ctx, int n, int* dst);
void prepare_system_geometry(System& s, const double* box_host, double rc_r, double rc_a,
                             double skin);
// Expand the list into the caller's numbering (see nep_get_neighbors).
hipError_t unpack_neighbors(nep_ctx ctx, int* nbr, int* img, int* cnt_r, int* cnt_a, int* rev);
// Reverse slots of a list (any system, global atom indices).
void launch_reverse(nep_ctx ctx, int n, int cap, const uint32_t* nl, const int* cnt_r,
                    const int* cnt_a, int* rev);

// force.hip
bool have_force_variant(const nep_hyper& h);
// The dataset (training, differentiation) kernels exist for the default sizes only.
bool have_training_variant(const nep_hyper& h);
// generic.hip: pass 1 for any size with n_max <= 15, l_max <= 4, <= 64 neurons
// (one wave per atom).
bool generic_supports(const nep_hyper& h);
hipError_t launch_partials_generic(nep_ctx ctx, const double* pos);
// pass 1: descriptor, network, partial forces; pass 2: scatter-free gather.
// Pass 1 on the internal system with tile shape `variant` (0, 1, 2 = 2, 4, 8
// lanes per atom, 3 = one wave per atom; -1 = the context's choice).  Models
// other than the default sizes always use the one-wave-per-atom kernel.
hipError_t launch_partials(nep_ctx ctx, const double* pos, int variant = -1);
// mode 0: plain evaluation (totals = E, W(9), J(3)); mode 1: velocity-Verlet
// second half-kick fused (vel updated, thermo row written).
// Pass 2 (k_gather, modes as documented there) writing per-block sums to
// block_out [gather_blocks(n)][13 or 5]; launch_finalize adds nsets such
// arrays (consecutive in block_sums) into out [nsets][nq].  fe [3]: the
// HNEMD driving field added as F_e . W_i in the MD modes.
hipError_t launch_gather(nep_ctx ctx, const double* pos, double* vel, float* U_out, float* F_out,
                         float* W_out, float* J_out, double* block_out, int mode, double kick,
                         double mass, double dt, double* pos_next, const double* fe, bool last);
hipError_t launch_finalize(nep_ctx ctx, int nq, int nsets, const double* block_sums, double* out,
                           bool first);
size_t gather_blocks(int n);
// The caller's positions and velocities (caller order) gathered into the
// internal arrays with the first half-kick and drift applied (the forces kept
// in the context belong to these positions).
hipError_t launch_take_kick_drift(nep_ctx ctx, const double* pos_c, const double* vel_c,
                                  double* pos, double* vel, double kick, double mass, double dt);
hipError_t launch_kick_drift(nep_ctx ctx, double* pos, double* vel, double kick, double mass,
                             double dt);
// pass 1 over a dataset for n_pop parameter vectors Z [n_pop][n_par].
hipError_t launch_partials_population(nep_ctx ctx, nep_dataset ds, int n_pop, const float* Z);

// backward.hip: parameter (and energy-part position) gradient over a dataset.
hipError_t launch_backward(nep_ctx ctx, nep_dataset ds, const float* z, const double* gE,
                           const float* gF, const float* F, double* gpos, double* grad,
                           float* grad32);

// Launch a kernel on the context's stream.  When a timed kernel class is
// being launched, its first kernel carries the start event and its last
// kernel the stop event in the dispatch itself (no extra packets).
template <typename F, typename... Args>
inline void launch_kernel(nep_ctx ctx, bool first, bool last, F kernel, dim3 grid, dim3 block,
                          Args... args) {
  hipEvent_t a = first ? ctx->ev_first : nullptr;
  hipEvent_t b = last ? ctx->ev_last : nullptr;
  if (a || b)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, ctx->stream, a, b, 0, args...);
  else
    kernel<<<grid, block, 0, ctx->stream>>>(args...);
}

// Run `launch` (which enqueues the kernels of class `cls`) with that class's
// timing events attached when timing is on.
template <class Fn>
hipError_t timed(nep_ctx ctx, int cls, Fn&& launch) {
  KernelTimer& t = ctx->timer;
  if (!t.on) return launch();
  if (t.used[cls] == t.start[cls].size()) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) {
      (void)hipEventDestroy(a);
      return e;
    }
    t.start[cls].push_back(a);
    t.stop[cls].push_back(b);
  }
  const size_t k = t.used[cls]++;
  ctx->ev_first = t.start[cls][k];
  ctx->ev_last = t.stop[cls][k];
  hipError_t e = launch();
  ctx->ev_first = ctx->ev_last = nullptr;
  return e;
}

// Make the context's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// helpers (nep_api.hip)
nep_status fail(nep_ctx ctx, nep_status code, const std::string& msg);
nep_status check_hip(nep_ctx ctx, hipError_t e, const char* what);
int n_des_of(const nep_hyper& h);
// One force evaluation of the internal state (positions sys.pos_s, velocities
// sys.vel_s when vel is true): pass 1 and pass 2 into the internal U, F, W, J,
// with the totals (13 values, or 5 thermo values in the MD modes) in out.
// MD modes: block sums go to block_out and are reduced later (out unused).
hipError_t evaluate_internal(nep_ctx ctx, bool vel, double* out, int mode, double kick,
                             double mass, bool want_w = false, bool want_j = false,
                             double* block_out = nullptr, double dt = 0.0,
                             double* pos_next = nullptr, const double* fe = nullptr);
// noalloc.hip: locate the static workspace of nep_evaluate_static on the
// current device (once per device, at context creation).
void scratch_setup(int device);
// Check a box and its list geometry for a neighbour build (as
// nep_build_neighbors does); fills `probe` on success.
nep_status check_box(nep_ctx ctx, const double* box_host, double skin, System& probe);

}  // namespace nep
