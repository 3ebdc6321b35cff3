/*
 * nep.h -- C ABI of libnep, the MI355X (gfx950) implementation of the hot
 * path of the neuroevolution potential (NEP) of Fan et al., arXiv 2107.08119:
 * per-atom Chebyshev radial and Legendre angular descriptors, a one-hidden-
 * layer tanh network, analytic partial forces, and from them forces, full
 * per-atom virials and heat currents, velocity-Verlet molecular dynamics and
 * the separable-NES population loss.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Plain C types only; no exception crosses the ABI.  Every call returns a
 *    nep_status; nep_last_error() gives a message for the last failure.
 *  - Array arguments are owned by the caller.  Names ending in _dev are
 *    device pointers (HBM of the context's device); names ending in _host
 *    are host pointers.  The library never frees caller memory.
 *  - The context owns its neighbour lists, partial forces and scratch; it
 *    never touches caller buffers outside a call's documented outputs.
 *  - Work is enqueued on the HIP stream given to nep_create (borrowed, not
 *    owned).  Calls return after argument checks, before the device work
 *    completes, except where stated.  Device-side failures (neighbour
 *    capacity, image range, non-finite energy) are latched in the context
 *    and reported by nep_synchronize() and by the next call that checks them.
 *  - Units: Angstrom, fs, amu, eV.  Forces in eV/A, virials in eV, heat
 *    currents in eV A/fs, velocities in A/fs.
 *  - Atom arrays are structure-of-arrays: positions and velocities are
 *    float64 [3][N] (all x, then all y, then all z); forces [3][N] float32;
 *    per-atom virials [9][N] float32 with component (a,b) at row 3a+b;
 *    heat currents [3][N] float32.
 *  - A box is 9 float64 host values: the three cell vectors as rows, so that
 *    a lattice translation is n0*a + n1*b + n2*c.
 *  - Pair displacement convention r_ij = r_j - r_i (paper, Sec. II A).
 */
#ifndef NEP_H_
#define NEP_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nep_ctx_s* nep_ctx;
typedef struct nep_dataset_s* nep_dataset;
typedef struct nep_vvcf_s* nep_vvcf;

typedef enum {
  NEP_OK = 0,
  NEP_EINVAL = 1,      /* bad argument (null pointer, size, layout)            */
  NEP_ESTATE = 2,      /* call order: parameters or neighbour list missing     */
  NEP_ENOMEM = 3,      /* device allocation failed                            */
  NEP_EOVERFLOW = 4,   /* an atom has more neighbours than max_neighbors      */
  NEP_ENONFINITE = 5,  /* a non-finite energy or force was produced           */
  NEP_EDEVICE = 6,     /* a HIP runtime call failed                           */
  NEP_ENOTIMPL = 7,    /* hyperparameters without a compiled kernel variant   */
  NEP_EIMAGE = 8,      /* a pair needs a lattice image beyond +-3 cells       */
  NEP_ESKIN = 9        /* an atom moved more than skin/2 since its list build */
} nep_status;

/* Hyperparameters of Table nep-hyper (Sec. III B): radial and angular cutoffs
 * r_c^R, r_c^A (A), Chebyshev orders n_max^R, n_max^A (n = 0..n_max), Legendre
 * order l_max (l = 1..l_max) and hidden neurons N_neu.  The descriptor has
 * N_des = (n_max^R+1) + (n_max^A+1) l_max components (Eq. N_des) and the
 * network N_par = (N_des+2) N_neu + 1 parameters (Eq. N_par).  Requires
 * 0 < rc_angular <= rc_radial.  Force evaluation and MD: (n_max^R, n_max^A,
 * l_max, N_neu) = (8, 4, 4, 30) has tuned kernels (2, 4 or 8 lanes per atom);
 * any n_max^R, n_max^A <= 15, 1 <= l_max <= 4, N_neu <= 64 (e.g. the paper's
 * 80-50-1 silicon model) runs on a one-wave-per-atom kernel; other sizes
 * return NEP_ENOTIMPL.  Datasets, SNES and the backward need (8, 4, 4, 30). */
typedef struct {
  double rc_radial, rc_angular;
  int n_max_radial, n_max_angular, l_max, n_neuron;
} nep_hyper;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t, or NULL for the null stream).  *out is set on success. */
nep_status nep_create(nep_ctx* out, int device, void* hip_stream);

/* Free everything the context owns.  Waits for its stream first.  NULL is ok. */
void nep_destroy(nep_ctx ctx);

/* Message of the last failure of a call on this context ("" if none).  The
 * string is owned by the context and valid until its next call. */
const char* nep_last_error(nep_ctx ctx);

/* Replace the stream used by later calls (borrowed). */
nep_status nep_set_stream(nep_ctx ctx, void* hip_stream);

/* Wait for all enqueued work; return the first latched device error
 * (NEP_EOVERFLOW, NEP_EIMAGE, NEP_ENONFINITE, NEP_ESKIN) and clear it, else
 * NEP_OK. */
nep_status nep_synchronize(nep_ctx ctx);

/* N_des and N_par of a hyperparameter set (Eqs. N_des, N_par); 0 if invalid. */
int nep_num_descriptors(const nep_hyper* hyper);
int nep_num_params(const nep_hyper* hyper);

/* ------------------------------------------------------------- the model */

/* Copy the parameter vector z (host, float32, n_par values) to the device.
 * Layout (Sec. II D): w1 [N_neu][N_des] row-major (w1[mu][nu] is the weight
 * from descriptor component nu to neuron mu), b1 [N_neu], w2 [N_neu], b2.
 * Descriptor order nu: radial n = 0..n_max^R, then angular components
 * (n, l) at N_R + n*l_max + (l-1).  Site energy
 *   U_i = sum_mu w2[mu] tanh(sum_nu w1[mu][nu] q_nu - b1[mu]) - b2
 * (Eqs. nn1, nn2).  NEP_EINVAL unless n_par == nep_num_params(hyper).
 * Synchronous with respect to the host buffer. */
nep_status nep_load_params(nep_ctx ctx, const nep_hyper* hyper, const float* z_host, int n_par);

/* ------------------------------------------------------------ neighbours */

/* Build the neighbour list of a periodic system of n_atoms atoms at pos_dev
 * ([3][N] float64).  An entry (j, n) of atom i is kept iff
 *   |r_j + n.H - r_i|^2 < (rc_radial + skin)^2
 * with the displacement and its squared norm evaluated in float64 as
 *   d_c = (x_jc - x_ic) + ((n0*H_0c + n1*H_1c) + n2*H_2c),
 *   |d|^2 = (d_x*d_x + d_y*d_y) + d_z*d_z          (no fused multiply-add),
 * and (j, n) != (i, 0) -- the paper's site environment within a cutoff
 * (Sec. II A).  Entries with |d|^2 < (rc_angular + skin)^2 come first in
 * each atom's list.  Every lattice image is a separate entry, so boxes
 * thinner than twice the cutoff are handled; images beyond +-3 cells latch
 * NEP_EIMAGE.  max_neighbors bounds the list length (more latches
 * NEP_EOVERFLOW).  n_atoms must be below 2^23 and max_neighbors * n_atoms
 * below 2^31.  Requires loaded parameters.  The library keeps its own copy of
 * the positions, re-sorted into cell order at every list build; results are
 * always returned in the caller's atom order. */
nep_status nep_build_neighbors(nep_ctx ctx, int n_atoms, const double* pos_dev,
                               const double* box_host, double skin, int max_neighbors);

/* Copy the current list to caller device buffers (for inspection):
 * cnt_radial_dev, cnt_angular_dev [N] int32; nbr_dev [max_neighbors][N] int32
 * holding j; img_dev [max_neighbors][N][3] int32 holding (n0, n1, n2)
 * (slot s of atom i at (s*N + i)*3); rev_dev [max_neighbors][N] int32 holding
 * the slot of the reverse entry (i, -n) in atom j's list.  Entries at
 * s >= cnt are unspecified.  Any pointer may be NULL. */
nep_status nep_get_neighbors(nep_ctx ctx, int* cnt_radial_dev, int* cnt_angular_dev,
                             int* nbr_dev, int* img_dev, int* rev_dev);

/* Multicomponent system (Sec. II C, multicomponent systems): atomic numbers
 * atomic_numbers_host [n] (caller order, 1..118) multiply the cutoff function
 * of every pair (i, j) by sqrt(Z_i Z_j), in the radial and angular terms
 * alike; one network serves every species.  masses_amu_host [n] (> 0, or
 * NULL) gives each atom its own mass in nep_md_step / nep_md_step_driven,
 * whose mass_amu is then only a reference value (still > 0).  n must equal
 * the atom count of the last nep_build_neighbors (NEP_ESTATE before any);
 * the arrays are copied (host memory, synchronous) and persist across list
 * rebuilds until a build with another atom count or a call with
 * atomic_numbers_host == NULL, which returns to one species with the mass of
 * each call.  With species set, forces come from the one-wave-per-atom
 * kernel (nep_autotune reports 64 lanes).  The training entry points
 * (datasets, SNES, backward) remain one-species.  NEP_EINVAL for n or a value
 * out of range. */
nep_status nep_set_species(nep_ctx ctx, int n, const int* atomic_numbers_host,
                           const double* masses_amu_host);

/* ------------------------------------------------------------ evaluation */

/* One force evaluation of the system last passed to nep_build_neighbors
 * (same n_atoms and box; positions may have moved by at most skin/2: an
 * evaluation that finds an atom farther than skin/2 from its position at the
 * list build, compared in float32, latches NEP_ESKIN, since the list may then
 * miss pairs inside the cutoff).
 * Computes, per Sec. II A-D:
 *   U_i (site energy), F_i = sum_j (dU_i/dr_ij - dU_j/dr_ji),
 *   W_i = sum_j r_ij (x) dU_j/dr_ji (full 3x3, Eq. Wi), J_i = W_i . v_i,
 * in float32 arithmetic with float64 positions and float64 totals.
 * Outputs (any may be NULL except F_dev): U_dev [N], F_dev [3][N],
 * W_dev [9][N], J_dev [3][N] (needs vel_dev [3][N] float64), totals_dev
 * [13] float64 = (sum U, sum W (9, row-major), sum J (3)). */
nep_status nep_compute(nep_ctx ctx, const double* pos_dev, const double* vel_dev, float* U_dev,
                       float* F_dev, float* W_dev, float* J_dev, double* totals_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the work of
 * nep_build_neighbors followed by nep_compute in one call that makes no
 * hipMalloc, hipFree or other allocation.  The neighbour list, partial forces
 * and block sums live in a static workspace of nep_static_workspace_bytes()
 * bytes (32 MiB) on each device, reserved while the library is loaded there
 * and located at nep_create.
 *   n_atoms, pos_dev [3][N] float64, box_host [9] (rows a, b, c in Angstrom,
 *   host), skin, max_neighbors: as for nep_build_neighbors;
 *   vel_dev [3][N] float64 or NULL; U_dev [N], F_dev [3][N], W_dev [9][N],
 *   J_dev [3][N] float32 and totals_dev [13] float64: as for nep_compute
 *   (F_dev required; J_dev needs vel_dev; totals_dev NULL keeps the totals in
 *   the context).
 * The context's parameters and stream are used; its own neighbour list,
 * species, masses and the MD state kept by nep_md_step are left as they
 * were.  One species (nep_set_species does not apply).  All arrays are
 * caller-owned; nothing is kept after the call except in the workspace.
 * NEP_EINVAL when the system needs more than the workspace (about
 * 36 * max_neighbors + 300 bytes per atom, plus 12 bytes per list cell; e.g.
 * 8,000 atoms with 64 slots fit) and for the arguments nep_build_neighbors
 * rejects; NEP_EDEVICE if the workspace could not be located on this device.
 * Device errors (list overflow, non-finite values) are latched as for the
 * other calls and reported by nep_synchronize.  Every call on one device
 * shares its workspace, which keeps the last call's contents: calls that
 * overlap on one GPU (different streams or host threads) race. */
nep_status nep_evaluate_static(nep_ctx ctx, int n_atoms, const double* pos_dev,
                               const double* box_host, double skin, int max_neighbors,
                               const double* vel_dev, float* U_dev, float* F_dev, float* W_dev,
                               float* J_dev, double* totals_dev);

/* Size in bytes of the per-device static workspace of nep_evaluate_static. */
size_t nep_static_workspace_bytes(void);

/* n_steps of velocity-Verlet NVE for atoms of mass mass_amu:
 *   v += dt/2 F/m;  r += dt v;  (rebuild the list every rebuild_every steps,
 *   first wrapping positions into the box);  F = F(r);  v += dt/2 F/m.
 * pos_dev, vel_dev: [3][N] float64, updated in place.  thermo_dev
 * [n_steps][5] float64 receives per step (E_pot, E_kin, sum J_x, J_y, J_z)
 * evaluated with the end-of-step velocities.  W_dev [9][N] / J_dev [3][N]
 * (float32, may be NULL) receive the per-atom virial and heat current at
 * every step (so they hold the last step's on return).  Requires a prior
 * nep_build_neighbors for this system (its skin and max_neighbors are
 * reused).  Forces of the starting positions are computed first unless the
 * previous call was nep_md_step on the same buffers.  Every step checks that
 * no atom has moved more than skin/2 since the list in use was built; a
 * violation (rebuild_every too long for the skin and the dynamics) latches
 * NEP_ESKIN, reported by nep_synchronize: the trajectory may then have missed
 * pairs and should be rerun with a shorter interval or a larger skin. */
nep_status nep_md_step(nep_ctx ctx, int n_steps, double dt_fs, int rebuild_every,
                       double mass_amu, double* pos_dev, double* vel_dev, double* thermo_dev,
                       float* W_dev, float* J_dev);

/* nep_md_step with the homogeneous driving force of the HNEMD method (Sec.
 * II B): every atom also feels F_i^ext = F_e . W_i, i.e.
 * (F_i^ext)_b = sum_a fe_host[a] (W_i)_ab, with W_i the per-atom virial of the
 * same step (fe_host [3] in 1/Angstrom, host memory).  The energy then grows
 * at the rate F_e . J.  fe = (0, 0, 0) is nep_md_step.  The forces kept for
 * the next call include the driving force of this call's F_e. */
nep_status nep_md_step_driven(nep_ctx ctx, int n_steps, double dt_fs, int rebuild_every,
                              double mass_amu, const double* fe_host, double* pos_dev,
                              double* vel_dev, double* thermo_dev, float* W_dev, float* J_dev);

/* ------------------------------------------ spectral heat transport */

/* Virial-velocity correlation of an HNEMD run (Sec. II B):
 *   K_mu(t) = sum_i < sum_nu (W_i(0))_mu,nu (v_i(t))_nu >,
 * averaged over every time origin of the sampled trajectory, for lags
 * t = 0 .. n_lags-1 sample intervals.  The last n_lags samples' per-atom
 * virials are kept on the device (n_lags * 9 * n_atoms float32, at most
 * 64 GB).  *out owns them until nep_vvcf_destroy.  NEP_EINVAL for sizes out
 * of range. */
nep_status nep_vvcf_create(nep_ctx ctx, int n_atoms, int n_lags, nep_vvcf* out);
void nep_vvcf_destroy(nep_vvcf v);

/* Add one sample: W_dev [9][N] float32 per-atom virials ((W_i)_ab at row
 * 3a+b, as written by nep_md_step) and vel_dev [3][N] float64 velocities of
 * the same instant, both in the caller's order, on the device.  Every lag
 * k <= min(samples, n_lags-1) gains the term of origin (this sample - k).
 * Sums are float64, in a fixed order.  Asynchronous on the context's stream. */
nep_status nep_vvcf_sample(nep_ctx ctx, nep_vvcf v, const float* W_dev, const double* vel_dev);

/* The averaged correlation K_host [n_lags][3] (eV A/fs; lags with no
 * origin yet are 0) and the number of samples (either may be NULL).
 * Synchronous. */
nep_status nep_vvcf_get(nep_ctx ctx, nep_vvcf v, double* K_host, long long* samples);

/* Spectral conductivity from (2/TV) int K_mu(t) e^{i w t} dt = kappa_mu(w) F_e
 * for a driving force of magnitude fe (1/A) along one axis, samples dt_fs
 * apart, temperature (K) and volume (A^3): K is taken even in t, windowed by
 * (1 + cos(pi k / (n_lags-1)))/2 and summed by the trapezoid rule.  At the
 * n_nu frequencies nu_thz_host (THz, w = 2 pi nu): kappa_host [3][n_nu] in
 * W/(m K THz) (so int_0^inf kappa d nu is the conductivity in W/(m K)) and,
 * if not NULL, the quantum-corrected kappa_q_host [3][n_nu] =
 * kappa x^2 e^x / (e^x - 1)^2 with x = hbar w / k_B T (the correction of
 * Sec. IV C for disordered materials).  Host arrays; synchronous.
 * NEP_ESTATE before the first sample. */
nep_status nep_vvcf_spectrum(nep_ctx ctx, nep_vvcf v, double dt_fs, double temperature,
                             double volume, double fe, int n_nu, const double* nu_thz_host,
                             double* kappa_host, double* kappa_q_host);

/* ---------------------------------------------------- training (SNES) */

/* Copy a training set to the device and build its neighbour lists once
 * (Sec. II E; small structures are concatenated into one system, Sec. II F).
 * n_struct periodic cells; structure s has n_atoms_host[s] >= 1 atoms whose
 * positions follow those of structure s-1 in pos_host ([sum N][3] float64,
 * A), with cell vectors boxes_host[s] (9 float64, rows).  Targets: total
 * energy energy_host[s] (eV), forces forces_host ([sum N][3], eV/A), total
 * virial virial_host[s] (6 float64: xx yy zz xy yz zx, eV) used only when
 * has_virial_host[s] != 0.  Positions are wrapped into their cells on the
 * device.  Every lattice image within rc_radial (no skin) is a neighbour;
 * more than max_neighbors returns NEP_EOVERFLOW, cells thinner than half the
 * radial cutoff NEP_EINVAL.  Uses the hyperparameters of the last
 * nep_load_params.  All host arrays are read before the call returns;
 * *out owns device copies until nep_dataset_destroy. */
nep_status nep_dataset_create(nep_ctx ctx, int n_struct, const int* n_atoms_host,
                              const double* boxes_host, const double* pos_host,
                              const double* energy_host, const double* forces_host,
                              const double* virial_host, const unsigned char* has_virial_host,
                              int max_neighbors, nep_dataset* out);

/* Ordered pairs (i, j) of the dataset with r_ij inside the radial cutoff,
 * and inside the angular cutoff, counted when the dataset's geometry was
 * last prepared (creation or nep_dataset_set_positions).  Host only: makes
 * no device call.  NEP_EINVAL on a NULL argument. */
nep_status nep_dataset_pairs(nep_dataset ds, long long* radial_pairs, long long* angular_pairs);

/* Free a dataset (waits for its context's stream).  NULL is ok. */
void nep_dataset_destroy(nep_dataset ds);

/* Loss of n_pop parameter vectors (Eq. loss): Z_dev [n_pop][N_par] float32
 * on the device (layout as in nep_load_params); lambda_host = (lambda_e,
 * lambda_f, lambda_v, lambda_1, lambda_2).  Writes loss_dev [n_pop][6]
 * float64 = (L, L_e, L_f, L_v, L_1, L_2) with
 *   L_e = sqrt(mean_s ((U_s - E_s)/N_s)^2),
 *   L_f = sqrt(sum_i |F_i - F_i^tar|^2 / (3 N)),
 *   L_v = sqrt(sum_{s with virial} sum_6 ((W_s - W_s^tar)/N_s)^2 / (6 N_v)),
 *   L_1 = mean |z|,  L_2 = sqrt(mean z^2),
 * where U_s and W_s = sum_i W_i are the NEP energy and virial of structure s.
 * All individuals are evaluated by the same two launches, on the matrix
 * cores: the network and dU/dq of every (individual, atom), then one block
 * per tile of whole structures that contracts the descriptor derivatives
 * cached when the dataset's positions were set (Sec. II D) with every
 * individual's dU/dq, gathers the forces in LDS and forms the squared errors.
 * Forces and structure virials are summed as 32-bit fixed point, round(x 2^e)
 * with e per (tile of structures, individual) chosen from a bound on
 * |dU/dq| so that no sum reaches 2^30 (each term then carries an absolute
 * error of at most 2^-e-1, at most 2^-30 of the bound); integer sums do not depend on
 * their order.  The squared errors are float64 sums in a fixed order.  The
 * result of an individual does not depend on the rest of the population, and
 * a non-finite bound gives NaN losses.  The network kernel uses the shape
 * chosen by snes_autotune (32 atoms per wave until then).  The dataset must
 * belong to ctx and match its hyperparameters.  NEP_EINVAL if a structure has
 * more than 13,312 atoms (the forces of one individual on one structure must
 * fit in 160 KB of LDS); more than 52 individuals per 256-atom structure
 * take one more contraction launch per 52. */
nep_status snes_eval_population(nep_ctx ctx, nep_dataset ds, int n_pop, const float* Z_dev,
                                const double* lambda_host, double* loss_dev);

/* Tile-shape autotuner for snes_eval_population on this dataset: times each
 * compiled shape of the network kernel (16, 32 and 64 atoms per wave, i.e.
 * weight fragments reused over 1, 2 or 4 matrix tiles) over `reps`
 * evaluations (1..1000) of Z_dev [n_pop][N_par] with HIP events on the
 * context's stream, and keeps the fastest for later calls on the dataset.
 * Host outputs (either may be NULL): *atoms_out = chosen atoms per wave;
 * ms_out[3] = mean ms per evaluation of the shapes in the order above.
 * Waits for the stream. */
nep_status snes_autotune(nep_ctx ctx, nep_dataset ds, int n_pop, const float* Z_dev, int reps,
                         int* atoms_out, double* ms_out);

/* Use `atoms` (16, 32 or 64) atoms per wave in the network kernel of this
 * dataset, e.g. to reproduce a tuned choice.  NEP_EINVAL for other values. */
nep_status snes_set_tile(nep_ctx ctx, nep_dataset ds, int atoms);

/* Draw the population of generation `generation` (Sec. II E 2, step 2a):
 * r_dev [n_pop][n_par] standard normal (float32) and Z_dev = m + s . r
 * (float32, rounded from float64), with m_dev, s_dev [n_par] float32.  Noise
 * for individual k, parameters 4b..4b+3: Philox-4x32-10 (Salmon et al.,
 * SC'11) of counter (b, k, generation, 0) and key (seed low 32 bits, seed
 * high 32 bits), uniforms u = (x + 1/2) 2^-32, Box-Muller on (u0, u1) and
 * (u2, u3) in float64. */
nep_status snes_sample(nep_ctx ctx, int n_par, int n_pop, const float* m_dev, const float* s_dev,
                       unsigned long long seed, int generation, float* r_dev, float* Z_dev);

/* SNES update (Sec. II E 2, steps 2b-2d): rank individuals by loss_dev[k*6]
 * (ascending; NaN ranks last; ties by index), rank utilities
 * u_k = max(0, ln(P/2+1) - ln k) / sum_j max(0, ln(P/2+1) - ln j) - 1/P,
 * grad_m = sum_k u_k r_k, grad_s = sum_k u_k (r_k^2 - 1) summed in rank order
 * in float64, then m += eta_m s . grad_m and s *= exp(eta_s/2 grad_s) in
 * float64, stored as float32 in place.  eta_m <= 0 selects 1 and eta_s <= 0
 * selects (3 + ln n_par) / (5 sqrt(n_par)).  1 <= n_pop <= 1024. */
nep_status snes_update(nep_ctx ctx, int n_par, int n_pop, float* m_dev, float* s_dev,
                       const float* r_dev, const double* loss_dev, double eta_m, double eta_s);

/* n_gen generations of SNES on the device (Sec. II E 2): generation g =
 * generation .. generation + n_gen - 1 runs snes_sample (seed, g),
 * snes_eval_population and snes_update exactly as the separate calls do,
 * with m_dev, s_dev [n_par] updated in place and r_dev, Z_dev
 * [n_pop][n_par], loss_dev [n_pop][6] as their workspaces (they hold the last
 * generation's values afterwards).  best_dev [n_gen][6] (float64, may be
 * NULL) receives the loss terms of each generation's best individual (NaN
 * ranks last, ties by index).  The generation's launches are captured once
 * into a HIP graph and replayed n_gen times on the context's stream; the
 * generation counter lives in device memory, so nothing returns to the host
 * between generations.  The graph is kept for the next call with the same
 * arguments.  n_par must equal N_par of the loaded hyperparameters;
 * 1 <= n_pop <= 1024. */
nep_status snes_run(nep_ctx ctx, nep_dataset ds, int n_par, int n_pop, float* m_dev,
                    float* s_dev, unsigned long long seed, int generation, int n_gen,
                    const double* lambda_host, double eta_m, double eta_s, float* r_dev,
                    float* Z_dev, double* loss_dev, double* best_dev);

/* -------------------------------------------------------- differentiation */

/* Replace the positions of a dataset's atoms (pos_dev [3][sum N] float64 on
 * the device, same order and structures as at creation), wrap them into their
 * cells and rebuild the lists.  NEP_EOVERFLOW if a list outgrows its capacity. */
nep_status nep_dataset_set_positions(nep_ctx ctx, nep_dataset ds, const double* pos_dev);

/* Copy the dataset's current (wrapped) positions to pos_dev [3][sum N]. */
nep_status nep_dataset_get_positions(nep_ctx ctx, nep_dataset ds, double* pos_dev);

/* Forward evaluation of one parameter vector z_dev [N_par] (float32, device)
 * over a dataset: energy_dev [S] (E_s = sum_i U_i, float64), forces_dev
 * [3][sum N] (float32, Sec. II A), and, unless NULL, virial_dev [S][9]
 * (float64, sum_i W_i of each structure, row-major). */
nep_status nep_dataset_compute(nep_ctx ctx, nep_dataset ds, const float* z_dev,
                               double* energy_dev, float* forces_dev, double* virial_dev);

/* Backward of the dataset evaluation.  With gE_dev [S] (float64, may be NULL
 * for zero) and gF_dev [3][sum N] (float32, may be NULL for zero):
 *   grad_z_dev [N_par] (float64) = d/dz [ sum_s gE_s E_s + sum_i gF_i . F_i ],
 * the parameter gradient of an energy + force objective.  The force part is
 * the mixed second derivative sum_a sum_nu d(dU_a/dq_nu)/dz delta q_a,nu with
 * delta q_a = sum_j (dq_a/dr_aj) (gF_a - gF_j) (partial-force expressions of
 * Sec. II D applied to gF).  Unless NULL, grad_z32_dev [N_par] receives the
 * same values in float32 and grad_pos_dev [3][sum N] (float64) the position
 * gradient of the energy part, -gE_s F_i, which needs forces_dev from
 * nep_dataset_compute of the same z (the force part's position gradient,
 * which would need second derivatives, is not computed).  Sums are float64 in
 * a fixed order. */
nep_status nep_dataset_backward(nep_ctx ctx, nep_dataset ds, const float* z_dev,
                                const double* gE_dev, const float* gF_dev,
                                const float* forces_dev, double* grad_pos_dev,
                                double* grad_z_dev, float* grad_z32_dev);

/* ----------------------------------------------------------- measurement */

/* Kernel timing for benchmarks.  While enabled, every launch of the force
 * passes, the neighbour-list build and the integrator is bracketed by a pair
 * of HIP events recorded on the context's stream.  Disabled by default. */
nep_status nep_set_timing(nep_ctx ctx, int enable);

/* Waits for the stream, then returns per kernel class the summed event time
 * in milliseconds (ms_out[4]) and the number of launches (launches_out[4])
 * since timing was enabled or last read, and resets both.  Classes:
 * 0 descriptor/network/partial forces, 1 force/virial/heat-current gather,
 * 2 neighbour-list build, 3 integrator kick-drift. */
nep_status nep_get_timing(nep_ctx ctx, double* ms_out, int* launches_out);

/* Enqueue `reps` back-to-back launches of the descriptor/network/partial-
 * force kernel on the current system at pos_dev (each launch recomputes the
 * same outputs) between one pair of HIP events on the context's stream, wait
 * for them, and return the mean duration of one launch in milliseconds.
 * Needs loaded parameters and a neighbour list; 1 <= reps <= 100000. */
nep_status nep_time_partials(nep_ctx ctx, const double* pos_dev, int reps, double* ms_per_launch);

/* Tile-shape autotuner for the descriptor/network/partial-force kernel on
 * the current system at pos_dev (as for nep_compute): times the compiled
 * shapes (2, 4 and 8 lanes per atom; 128, 64 and 32 atoms per block) with
 * HIP events on the context's stream in three interleaved rounds of `reps`
 * launches per shape (1..10000), so that a clock that settles during the
 * calls weighs on every shape alike, and keeps the shape with the fastest
 * round for later nep_compute / nep_md_step calls.  Host outputs (either may
 * be NULL): *lanes_out = chosen lanes per atom; ms_out[3] = mean ms per
 * launch of each shape's fastest round, in the order above.  Needs loaded
 * parameters and a neighbour list; waits for the stream. */
nep_status nep_autotune(nep_ctx ctx, const double* pos_dev, int reps, int* lanes_out,
                        double* ms_out);

/* Use `lanes` (2, 4 or 8) lanes per atom in the descriptor/network/partial-
 * force kernel of this context, or 64 for the one-wave-per-atom kernel that
 * every model size uses.  NEP_EINVAL for other values. */
nep_status nep_set_tile(nep_ctx ctx, int lanes);

#ifdef __cplusplus
}
#endif

#endif /* NEP_H_ */
