// Force evaluation on gfx950: descriptor -> network -> partial forces (pass 1)
// and the scatter-free gather of forces, virials and heat currents (pass 2).
//
// Pass 1 works on L consecutive lanes per atom.  The lanes split the atom's
// pairs, accumulate partial descriptor sums, and combine them with DPP lane
// permutations, so every lane ends with the full descriptor.  The model's
// terms (factorised angular descriptor, network, partial force) are in
// nep_terms.h.
//
// Pass 1 also sums the atom's own partials, sum_j p_ij, stores every p_ij
// in the reverse slot of atom j's list (each slot is written exactly once)
// and, for systems up to kPairVectorMaxAtoms atoms, the pair vector r_ij in
// the atom's own slot.  Pass 2 then computes, per atom,
// F_i = sum_j p_ij - sum_j p_ji, W_i = sum_j r_ij (x) p_ji and J_i = W_i v_i
// (Sec. II A-B) from coalesced reads of its own slots (and, for larger
// systems, the neighbours' positions); no atomics touch forces and the result is
// reproducible bit for bit.  Totals are summed in float64 per block and the
// block sums are added in block order by a one-block kernel.
#include "nep_terms.h"

namespace nep {
namespace {

// Neighbour slots per atom staged in LDS by pass 1: 40 KB of staged pairs per
// block (at most 64, the width of the per-atom slot masks).
constexpr int stage_slots(int atoms_per_block) {
  return 2560 / atoms_per_block < 64 ? 2560 / atoms_per_block : 64;
}

// ------------------------------------------------------------------ pass 1
// Outputs: U[i]; fown[c*n + i] = sum_j dU_i/dr_ij (component c); and every
// partial force dU_i/dr_ij written to the reverse slot, pin[t*n + j] with
// t = rev[s*n + i], where atom j finds it as its incoming partial dU_i/dr_ij.
// With geo (systems of up to kPairVectorMaxAtoms atoms), the pair vector
// r_ij of every slot s of atom i goes to geo[s*n + i] (float32, as used
// here) for pass 2's virial.
// MULTI: every atom has its own cell (struct_of[i] indexes boxes[][9]).
// Population: blockIdx.y selects parameter vector k at zpar + k*zstride and
// its outputs at pin + k*pstride, fown + 3nk, U + nk.
template <int NR, int NA, int LMAX, int NNEU, int L, bool MULTI>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_partials(
    int n, const double* __restrict__ pos, const uint32_t* __restrict__ nl,
    const int* __restrict__ cnt_r, const int* __restrict__ cnt_a, const int* __restrict__ rev,
    Box box, const double* __restrict__ boxes, const int* __restrict__ struct_of,
    const float* __restrict__ zpar, size_t zstride, float rc_r, float rc_a,
    Partial3* __restrict__ pin, size_t pstride, float* __restrict__ fown, float* __restrict__ U,
    Partial3* __restrict__ geo) {
  constexpr int NLM = Model<NR, NA, LMAX>::kNLM;
  constexpr int NDES = Model<NR, NA, LMAX>::kNDES;
  __shared__ float4 sw4[NetRows<NDES, NNEU>::kFloat4];
  __shared__ float sb2;
  {
    const size_t pk = blockIdx.y;
    zpar += pk * zstride;
    pin += pk * pstride;
    fown += pk * 3 * (size_t)n;
    U += pk * (size_t)n;
  }
  load_net_rows<NDES, NNEU>(zpar, sw4, &sb2);

  // Stage the first KS slots of the block's atoms in LDS, keeping only
  // the pairs inside a cutoff, compacted per atom: first the pairs inside
  // r_c^A (angular partition of the list), then those inside r_c^R only.
  // Each entry holds the pair displacement (float32, formed in float64) and,
  // in .w, the index of the reverse slot where dU_i/dr_ij is written; a slot
  // whose pair lies beyond r_c^R gets its zero partial force written here.
  // Thread tid handles atom a = tid % APB at slots w, w + W, ... (w = tid / APB),
  // so list reads coalesce and every thread has several loads in flight.
  constexpr int APB = kBlock / L;  // atoms per block
  constexpr int KS = stage_slots(APB);
  constexpr int W = kBlock / APB;  // slots staged side by side
  constexpr int T = KS / W;        // slots per thread
  static_assert(KS % W == 0 && KS <= 64, "staging shape");
  __shared__ float4 sd[KS][APB];
  __shared__ unsigned long long smask[2][W][APB];  // [angular, radial-only][w][atom]
  __shared__ int scount[2][APB];
  __shared__ int slist[2][APB];  // list counts (radial, angular part) of the block's atoms
  __shared__ __align__(16) float snet[kBlock / 64][net_rows(L) * kNetX];  // network_mfma
  const float rcr2 = rc_r * rc_r, rca2 = rc_a * rc_a;
  {
    const int a = threadIdx.x % APB, w = threadIdx.x / APB;
    const int ia = (int)xcd_block(blockIdx.x, gridDim.x) * APB + a;
    const int cra = ia < n ? cnt_r[ia] : 0;
    const int caa = ia < n ? cnt_a[ia] : 0;
    const double* Ha = MULTI && ia < n ? boxes + 9 * (size_t)struct_of[ia] : box.h;
    const double xa = ia < n ? pos[ia] : 0.0, ya = ia < n ? pos[n + ia] : 0.0,
                 za = ia < n ? pos[2 * n + ia] : 0.0;
    // all loads first (clamped to valid addresses), so that the T slots'
    // list and position reads are in flight together
    uint32_t e[T];
    int rv[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int sl = w + t * W;
      const size_t idx = sl < cra ? (size_t)sl * n + ia : 0;
      e[t] = nl[idx];
      rv[t] = rev[idx];
    }
    double pj[T][3];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int j = w + t * W < cra ? (int)(e[t] & kAtomMask) : 0;
      pj[t][0] = pos[j];
      pj[t][1] = pos[n + j];
      pj[t][2] = pos[2 * n + j];
    }
    float4 v[T];
    unsigned long long ma = 0, mr = 0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int sl = w + t * W;
      float dx, dy, dz;
      image_displacement(e[t], pj[t][0], pj[t][1], pj[t][2], xa, ya, za, Ha, dx, dy, dz);
      const int dst = rv[t] * n + (int)(e[t] & kAtomMask);
      v[t] = make_float4(dx, dy, dz, __int_as_float(dst));
      const float r2 = pair_r2(dx, dy, dz);
      if (geo && sl < cra) geo[(size_t)sl * n + ia] = Partial3{dx, dy, dz};
      if (sl < cra) {
        if (sl < caa && r2 < rca2)
          ma |= 1ull << sl;
        else if (r2 < rcr2)
          mr |= 1ull << sl;
        else
          pin[(size_t)(unsigned)dst] = Partial3{0.f, 0.f, 0.f};
      }
    }
    smask[0][w][a] = ma;
    smask[1][w][a] = mr;
    __syncthreads();
    unsigned long long fa = 0, fr = 0;
#pragma unroll
    for (int u = 0; u < W; ++u) {
      fa |= smask[0][u][a];
      fr |= smask[1][u][a];
    }
    const int na = __popcll(fa);
    if (w == 0) {
      scount[0][a] = na;
      scount[1][a] = __popcll(fr);
      slist[0][a] = cra;
      slist[1][a] = caa;
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int sl = w + t * W;
      const unsigned long long bit = 1ull << sl, below = bit - 1;
      if (fa & bit)
        sd[__popcll(fa & below)][a] = v[t];
      else if (fr & bit)
        sd[na + __popcll(fr & below)][a] = v[t];
    }
  }
  __syncthreads();

  const int gid = (int)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int i = gid / L;
  const int lane = gid % L;
  const int la = threadIdx.x / L;
  const bool active = i < n;
  const int ii = active ? i : 0;
  const int cr = slist[0][la];  // zero for atoms past n
  const int ca = slist[1][la];
  const int n_ang = scount[0][la];              // staged pairs inside r_c^A
  const int n_in = n_ang + scount[1][la];       // staged pairs inside r_c^R
  const double xi = pos[ii], yi = pos[n + ii], zi = pos[2 * n + ii];
  const double* H = MULTI ? boxes + 9 * (size_t)struct_of[ii] : box.h;
  const float rcr_inv = 1.f / rc_r, rca_inv = 1.f / rc_a;
  // Work item k of this atom: k < n_in is staged pair k (angular when
  // k < n_ang); k >= n_in is list slot KS + (k - n_in), read from the
  // list and classified here.
  const int n_work = n_in + (cr > KS ? cr - KS : 0);
  auto pair = [&](int k, float& dx, float& dy, float& dz, int& dst, bool& ang, bool& rad) {
    if (k < n_in) {
      const float4 v = sd[k][la];
      dx = v.x;
      dy = v.y;
      dz = v.z;
      dst = __float_as_int(v.w);
      ang = k < n_ang;
      rad = true;
    } else {
      const int s = KS + (k - n_in);
      const size_t idx = (size_t)s * n + i;
      int j;
      displacement(nl[idx], pos, n, xi, yi, zi, H, j, dx, dy, dz);
      dst = rev[idx] * n + j;
      const float r2 = pair_r2(dx, dy, dz);
      ang = s < ca && r2 < rca2;
      rad = r2 < rcr2;
    }
  };

  float q[NDES];
  float c[NA][NLM];

  // descriptor sums over this lane's share of the pairs; the first work item
  // (a dummy pair when the lane has none) starts them
  {
    int dst = 0;
    bool ang = false, rad = false;
    float dx = 1.f, dy = 0.f, dz = 0.f;
    if (lane < n_work) pair(lane, dx, dy, dz, dst, ang, rad);
    pair_descriptor_first<NR, NA, LMAX>(dx, dy, dz, rad, ang, rcr_inv, rca_inv, q, c);
  }
  for (int k = lane + L; k < n_work; k += L) {
    int dst;
    bool ang, rad;
    float dx, dy, dz;
    pair(k, dx, dy, dz, dst, ang, rad);
    pair_descriptor<NR, NA, LMAX>(dx, dy, dz, rad, ang, rcr_inv, rca_inv, q, c);
  }
#pragma unroll
  for (int a = 0; a < NR; ++a) q[a] = group_sum<L>(q[a]);
  radial_finish<NR>(q);
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int m = 0; m < NLM; ++m) c[a][m] = group_sum<L>(c[a][m]);
  angular_invariants<NR, NA, LMAX>(c, q);

  float dq[NDES];
  float u;
  network_mfma<NDES, NNEU, L>(q, sw4, sb2, snet[threadIdx.x >> 6], dq, u);
  if (active && lane == 0) U[i] = u;
  angular_coefficients<NR, NA, LMAX>(dq, c);
  const float dqs = radial_dq_sum<NR>(dq);

  // partial forces p_ij = dU_i/dr_ij for this lane's pairs
  float fx = 0.f, fy = 0.f, fz = 0.f;
  for (int k = lane; k < n_work; k += L) {
    int dst;
    bool ang, rad;
    float dx, dy, dz;
    pair(k, dx, dy, dz, dst, ang, rad);
    if (geo && k >= n_in) geo[(size_t)(KS + (k - n_in)) * n + i] = Partial3{dx, dy, dz};
    float px, py, pz;
    pair_force<NR, NA, LMAX>(dx, dy, dz, rad, ang, rcr_inv, rca_inv, dq, dqs, c, px, py, pz);
    fx += px;
    fy += py;
    fz += pz;
    pin[(size_t)(unsigned)dst] = Partial3{px, py, pz};
  }
  fx = group_sum<L>(fx);
  fy = group_sum<L>(fy);
  fz = group_sum<L>(fz);
  if (active && lane == 0) {
    fown[i] = fx;
    fown[n + i] = fy;
    fown[2 * n + i] = fz;
  }
}

// ------------------------------------------------------------------ pass 2
// Per-block sums of NQ doubles, written to partials[block][NQ]; a second
// kernel adds the blocks in order (no device-scope fence in the hot kernel).
template <int NQ>
__device__ __forceinline__ void block_partials(double (&v)[NQ], double* __restrict__ partials,
                                               unsigned block) {
  __shared__ double sw[kBlock / 64][NQ];
  const double s = block_sum<NQ>(v, sw);
  if (threadIdx.x < NQ) partials[(size_t)block * NQ + threadIdx.x] = s;
}

// Block x reduces set x: out[x][q] = sum over blocks b (in order of b) of
// partials[x][b][q].
template <int NQ>
__global__ __launch_bounds__(kBlock) void k_finalize(int nblocks, const double* __restrict__ partials,
                                                      double* __restrict__ out,
                                                      int* __restrict__ flags) {
  __shared__ double sw[kBlock / 64][NQ];
  partials += (size_t)blockIdx.x * nblocks * NQ;
  out += (size_t)blockIdx.x * NQ;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] += partials[(size_t)b * NQ + q];
  const double tot = block_sum<NQ>(acc, sw);
  if (threadIdx.x < NQ) {
    out[threadIdx.x] = tot;
    if (!isfinite(tot)) flags[kFlagNonFinite] = 1;
  }
}

// MODE 0: evaluation -> block sums of (U, W_ab (9), J (3)).
// MODE 1: velocity-Verlet second half-kick v += kick F, then block sums of
//         (E_pot, E_kin, J (3)) with the kicked velocities.
// MODE 2: MODE 1, then the next step's first half-kick v += kick F and drift
//         pos_next = pos + dt v (a separate array: pos is still being read).
// GEO: r_ij from pass 1's pair vectors geo[s*n + i]; otherwise formed again
// from the list entry and the neighbour's position (the same float32 value).
template <int L, int MODE, bool GEO>
__global__ __launch_bounds__(kBlock) void k_gather(
    int n, int cap, const double* __restrict__ pos, double* __restrict__ vel,
    const uint32_t* __restrict__ nl, const Partial3* __restrict__ geo,
    const int* __restrict__ cnt_r, const Partial3* __restrict__ pin,
    const float* __restrict__ fown, const float* __restrict__ U, Box box,
    float* __restrict__ U_out,
    float* __restrict__ F, float* __restrict__ W, float* __restrict__ J, double kick,
    double ekin_factor, double dt,
    double* __restrict__ pos_next, float fe0, float fe1, float fe2,
    const double* __restrict__ mass_c, const int* __restrict__ perm, double mref,
    const float* __restrict__ pos_ref, float half_skin2, int* __restrict__ flags,
    double* __restrict__ partials) {
  const unsigned bx = xcd_block(blockIdx.x, gridDim.x);
  const int gid = (int)bx * blockDim.x + threadIdx.x;
  const int i = gid / L;
  const int lane = gid % L;
  const bool active = i < n;
  const int ii = active ? i : 0;
  const int cr = active ? cnt_r[i] : 0;
  const double xi = pos[ii], yi = pos[n + ii], zi = pos[2 * n + ii];
  const double* H = box.h;
  // the atom's own loads of the epilogue, issued before the slot loop
  const float fo0 = active ? fown[i] : 0.f, fo1 = active ? fown[n + i] : 0.f,
              fo2 = active ? fown[2 * n + i] : 0.f;
  const bool own = active && lane == 0;
  const float ui = own ? U[i] : 0.f;
  const float rx = own ? pos_ref[i] : 0.f, ry = own ? pos_ref[n + i] : 0.f,
              rz = own ? pos_ref[2 * n + i] : 0.f;
  const double vx0 = own && vel ? vel[i] : 0.0, vy0 = own && vel ? vel[n + i] : 0.0,
               vz0 = own && vel ? vel[2 * n + i] : 0.0;
  const double mi = own && mass_c ? mass_c[perm[i]] : mref;
  float f0 = 0.f, f1 = 0.f, f2 = 0.f;
  float w[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) w[k] = 0.f;
  // B slots per lane at a time, all their loads issued before any use
  // (measured best on the 64,000-atom step: 9 of 9, 13, 17 with pair vectors
  // and 2 lanes per atom; 5 of 3, 5, 7, 9 otherwise with 4 lanes)
  constexpr int B = GEO && L == 2 ? 9 : 5;
  // The first batch is requested before the atom's slot count arrives: its
  // addresses need only the list capacity (every atom has cap rows; slots at
  // or past the count are read and not used).  Later batches stop at the count.
  int s0 = lane;
  do {
    const int bound = s0 == lane ? cap : cr;
    Partial3 rg[B], p[B];
    uint32_t e[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int s = s0 + u * L;
      const size_t idx = s < bound ? (size_t)s * n + ii : (size_t)ii;  // slot 0 past the end
      if constexpr (GEO)
        rg[u] = geo[idx];
      else
        e[u] = nl[idx];
      p[u] = pin[idx];
    }
    double pj[B][3];
    if constexpr (!GEO) {
#pragma unroll
      for (int u = 0; u < B; ++u) {
        // an entry past the count may be stale: its neighbour is not read
        const int j = s0 + u * L < cr ? (int)(e[u] & kAtomMask) : ii;
        pj[u][0] = pos[j];
        pj[u][1] = pos[n + j];
        pj[u][2] = pos[2 * n + j];
      }
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      if (s0 + u * L >= cr) break;
      float dx, dy, dz;
      if constexpr (GEO) {
        dx = rg[u].x;
        dy = rg[u].y;
        dz = rg[u].z;
      } else {
        image_displacement(e[u], pj[u][0], pj[u][1], pj[u][2], xi, yi, zi, H, dx, dy, dz);
      }
      const Partial3 pji = p[u];
      f0 -= pji.x;
      f1 -= pji.y;
      f2 -= pji.z;
      w[0] += dx * pji.x;
      w[1] += dx * pji.y;
      w[2] += dx * pji.z;
      w[3] += dy * pji.x;
      w[4] += dy * pji.y;
      w[5] += dy * pji.z;
      w[6] += dz * pji.x;
      w[7] += dz * pji.y;
      w[8] += dz * pji.z;
    }
    s0 += B * L;
  } while (s0 < cr);
  f0 = group_sum<L>(f0) + fo0;
  f1 = group_sum<L>(f1) + fo1;
  f2 = group_sum<L>(f2) + fo2;
#pragma unroll
  for (int k = 0; k < 9; ++k) w[k] = group_sum<L>(w[k]);
  if constexpr (MODE >= 1) {  // HNEMD driving force F_e . W_i (zero without a field)
    f0 += fe0 * w[0] + fe1 * w[3] + fe2 * w[6];
    f1 += fe0 * w[1] + fe1 * w[4] + fe2 * w[7];
    f2 += fe0 * w[2] + fe1 * w[5] + fe2 * w[8];
  }

  constexpr int NQ = MODE == 0 ? 13 : 5;
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  if (active && lane == 0) {
    // the list holds every pair within the cutoff only while no atom has
    // moved more than skin/2 since it was built (compared in float32, so an
    // unmoved atom gives exactly zero)
    const float ex = (float)xi - rx, ey = (float)yi - ry, ez = (float)zi - rz;
    if (ex * ex + ey * ey + ez * ez > half_skin2) flags[kFlagSkin] = 1;
    F[i] = f0;
    F[n + i] = f1;
    F[2 * n + i] = f2;
    if (U_out) U_out[i] = ui;
    if (W)
#pragma unroll
      for (int k = 0; k < 9; ++k) W[(size_t)k * n + i] = w[k];
    double vx = 0.0, vy = 0.0, vz = 0.0;
    // per-atom mass (caller order): the kick and kinetic factors were formed
    // for mass mref
    double ki = kick, ekf = ekin_factor;
    if (mass_c) {
      ki = kick * (mref / mi);
      ekf = ekin_factor * (mi / mref);
    }
    if (vel) {
      vx = vx0;
      vy = vy0;
      vz = vz0;
      if constexpr (MODE >= 1) {
        vx += ki * (double)f0;
        vy += ki * (double)f1;
        vz += ki * (double)f2;
        if constexpr (MODE == 1) {
          vel[i] = vx;
          vel[n + i] = vy;
          vel[2 * n + i] = vz;
        } else {
          const double ux = vx + ki * (double)f0, uy = vy + ki * (double)f1,
                       uz = vz + ki * (double)f2;
          vel[i] = ux;
          vel[n + i] = uy;
          vel[2 * n + i] = uz;
          pos_next[i] = xi + dt * ux;
          pos_next[n + i] = yi + dt * uy;
          pos_next[2 * n + i] = zi + dt * uz;
        }
      }
    }
    const double j0 = (double)w[0] * vx + (double)w[1] * vy + (double)w[2] * vz;
    const double j1 = (double)w[3] * vx + (double)w[4] * vy + (double)w[5] * vz;
    const double j2 = (double)w[6] * vx + (double)w[7] * vy + (double)w[8] * vz;
    if (J) {
      J[i] = (float)j0;
      J[n + i] = (float)j1;
      J[2 * n + i] = (float)j2;
    }
    v[0] = (double)ui;
    if constexpr (MODE == 0) {
#pragma unroll
      for (int k = 0; k < 9; ++k) v[1 + k] = (double)w[k];
      v[10] = j0;
      v[11] = j1;
      v[12] = j2;
    } else {
      v[1] = ekf * (vx * vx + vy * vy + vz * vz);
      v[2] = j0;
      v[3] = j1;
      v[4] = j2;
    }
  }
  block_partials<NQ>(v, partials, bx);
}

__global__ void k_kick_drift(int n, double* __restrict__ pos, double* __restrict__ vel,
                             const float* __restrict__ F, double kick, double dt,
                             const double* __restrict__ mass_c, const int* __restrict__ perm,
                             double mref) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * n) return;
  const double k = mass_c ? kick * (mref / mass_c[perm[t % n]]) : kick;
  const double v = vel[t] + k * (double)F[t];
  vel[t] = v;
  pos[t] += dt * v;
}

// k_kick_drift reading the caller's arrays: internal index k takes caller
// row perm[k] (the same arithmetic, so the same bits as a gather followed by
// k_kick_drift).
__global__ void k_take_kick_drift(int n, const double* __restrict__ pos_c,
                                  const double* __restrict__ vel_c, double* __restrict__ pos,
                                  double* __restrict__ vel, const float* __restrict__ F,
                                  double kick, double dt, const double* __restrict__ mass_c,
                                  const int* __restrict__ perm, double mref) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * n) return;
  const int k = t % n, r = t / n;
  const int c = perm[k];
  const double kk = mass_c ? kick * (mref / mass_c[c]) : kick;
  const double v = vel_c[(size_t)r * n + c] + kk * (double)F[t];
  vel[t] = v;
  pos[t] = pos_c[(size_t)r * n + c] + dt * v;
}

__global__ void k_zero_d(double* __restrict__ a, int m) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) a[t] = 0.0;
}

constexpr int kLanes = 4;  // lanes per atom

inline bool is_default_variant(const nep_hyper& h) {
  return h.n_max_radial == 8 && h.n_max_angular == 4 && h.l_max == 4 && h.n_neuron == 30;
}

inline unsigned blocks_for(size_t work, int block) { return (unsigned)((work + block - 1) / block); }

}  // namespace

bool have_force_variant(const nep_hyper& h) { return is_default_variant(h) || generic_supports(h); }

bool have_training_variant(const nep_hyper& h) { return is_default_variant(h); }

// Pass-2 tile: 2 lanes per atom with pair vectors from pass 1 on systems of
// 2^15 atoms or more, else 4 (the fastest of 1, 2, 4, 8 and 16 on the
// 64,000-atom step for each source of r_ij; below 2^15 atoms 4 lanes give
// the launch more waves, 1-2% faster on the 6,000-8,000-atom cells).
inline int gather_lanes(int n) { return n >= (1 << 15) && n <= kPairVectorMaxAtoms ? 2 : 4; }

size_t gather_blocks(int n) { return blocks_for((size_t)n * gather_lanes(n), kBlock); }

template <int L>
void launch_partials_shape(nep_ctx ctx, const double* pos, bool first, bool last) {
  const System& s = ctx->sys;
  const unsigned nb = blocks_for((size_t)s.n * L, kBlock);
  launch_kernel(ctx, first, last, k_partials<9, 5, 4, 30, L, false>, dim3(nb), dim3(kBlock), s.n,
                pos, (const uint32_t*)s.nl.ptr, (const int*)s.cnt_r.ptr, (const int*)s.cnt_a.ptr,
                (const int*)s.rev.ptr, s.box, (const double*)nullptr, (const int*)nullptr,
                (const float*)ctx->z.ptr, (size_t)0, (float)ctx->hyper.rc_radial,
                (float)ctx->hyper.rc_angular, ctx->p.ptr, (size_t)0, ctx->fown.ptr, ctx->U.ptr,
                s.n <= kPairVectorMaxAtoms ? ctx->geo.ptr : (Partial3*)nullptr);
}

hipError_t launch_partials(nep_ctx ctx, const double* pos, int variant) {
  const System& s = ctx->sys;
  if (s.n == 0) return hipSuccess;
  if (variant < 0) variant = ctx->md_variant;
  if (!is_default_variant(ctx->hyper) || variant == 3 || ctx->species_on())
    return launch_partials_generic(ctx, pos);
  switch (variant) {
    case 0:
      launch_partials_shape<2>(ctx, pos, true, true);
      break;
    case 2:
      launch_partials_shape<8>(ctx, pos, true, true);
      break;
    default:
      launch_partials_shape<4>(ctx, pos, true, true);
  }
  return hipGetLastError();
}

hipError_t launch_partials_population(nep_ctx ctx, nep_dataset ds, int n_pop, const float* Z) {
  if (ds->N == 0 || n_pop == 0) return hipSuccess;
  const unsigned nb = blocks_for((size_t)ds->N * kLanes, kBlock);
  launch_kernel(ctx, true, true, k_partials<9, 5, 4, 30, kLanes, true>, dim3(nb, n_pop),
                dim3(kBlock), ds->N, (const double*)ds->pos.ptr, (const uint32_t*)ds->nl.ptr,
                (const int*)ds->cnt_r.ptr, (const int*)ds->cnt_a.ptr, (const int*)ds->rev.ptr,
                Box{}, (const double*)ds->boxes.ptr, (const int*)ds->struct_of.ptr, Z,
                (size_t)ctx->n_par, (float)ctx->hyper.rc_radial, (float)ctx->hyper.rc_angular,
                ds->pin.ptr, (size_t)ds->cap * ds->N, ds->fown.ptr, ds->U.ptr,
                (Partial3*)nullptr);
  return hipGetLastError();
}

hipError_t launch_gather(nep_ctx ctx, const double* pos, double* vel, float* U_out, float* F_out,
                         float* W_out, float* J_out, double* block_out, int mode, double kick,
                         double mass, double dt, double* pos_next, const double* fe, bool last) {
  const System& s = ctx->sys;
  if (s.n == 0) return hipSuccess;
  const unsigned nb = (unsigned)gather_blocks(s.n);
  const double ekin_factor = 0.5 * mass / kAccel;
  const bool use_geo = s.n <= kPairVectorMaxAtoms;  // pass 1 wrote the pair vectors
  const uint32_t* nl = s.nl.ptr;
  const Partial3* geo = ctx->geo.ptr;
  const int* cnt = s.cnt_r.ptr;
  const Partial3* p = ctx->p.ptr;
  const float* fown = ctx->fown.ptr;
  const float* U = ctx->U.ptr;
  const bool per_atom = ctx->species_on() && ctx->have_masses;
  const double* mass_c = per_atom ? (const double*)ctx->masses.ptr : (const double*)nullptr;
  const float half_skin = (float)(0.5 * s.skin);
  auto go = [&](auto kernel) {
    launch_kernel(ctx, true, last, kernel, dim3(nb), dim3(kBlock), s.n, s.cap, pos, vel, nl, geo,
                  cnt, p,
                  fown, U, s.box, U_out, F_out, W_out, J_out, kick, ekin_factor, dt, pos_next,
                  (float)fe[0], (float)fe[1], (float)fe[2], mass_c, (const int*)s.perm.ptr, mass,
                  (const float*)s.pos_ref.ptr, half_skin * half_skin, ctx->flags.ptr, block_out);
  };
  if (use_geo && gather_lanes(s.n) == 2) {
    if (mode == 0)
      go(k_gather<2, 0, true>);
    else if (mode == 1)
      go(k_gather<2, 1, true>);
    else
      go(k_gather<2, 2, true>);
  } else if (use_geo) {
    if (mode == 0)
      go(k_gather<4, 0, true>);
    else if (mode == 1)
      go(k_gather<4, 1, true>);
    else
      go(k_gather<4, 2, true>);
  } else {
    if (mode == 0)
      go(k_gather<kLanes, 0, false>);
    else if (mode == 1)
      go(k_gather<kLanes, 1, false>);
    else
      go(k_gather<kLanes, 2, false>);
  }
  return hipGetLastError();
}

hipError_t launch_finalize(nep_ctx ctx, int nq, int nsets, const double* block_sums, double* out,
                           bool first) {
  if (nsets == 0) return hipSuccess;
  const int nb = (int)gather_blocks(ctx->sys.n);
  if (nq == 13)
    launch_kernel(ctx, first, true, k_finalize<13>, dim3(nsets), dim3(kBlock), nb, block_sums, out,
                  ctx->flags.ptr);
  else
    launch_kernel(ctx, first, true, k_finalize<5>, dim3(nsets), dim3(kBlock), nb, block_sums, out,
                  ctx->flags.ptr);
  return hipGetLastError();
}

hipError_t launch_take_kick_drift(nep_ctx ctx, const double* pos_c, const double* vel_c,
                                  double* pos, double* vel, double kick, double mass, double dt) {
  const int n = ctx->sys.n;
  if (n == 0) return hipSuccess;
  const bool per_atom = ctx->species_on() && ctx->have_masses;
  launch_kernel(ctx, true, true, k_take_kick_drift, dim3(blocks_for((size_t)3 * n, kBlock)),
                dim3(kBlock), n, pos_c, vel_c, pos, vel, (const float*)ctx->F.ptr, kick, dt,
                per_atom ? (const double*)ctx->masses.ptr : (const double*)nullptr,
                (const int*)ctx->sys.perm.ptr, mass);
  return hipGetLastError();
}

hipError_t launch_kick_drift(nep_ctx ctx, double* pos, double* vel, double kick, double mass,
                             double dt) {
  const int n = ctx->sys.n;
  if (n == 0) return hipSuccess;
  const bool per_atom = ctx->species_on() && ctx->have_masses;
  launch_kernel(ctx, true, true, k_kick_drift, dim3(blocks_for((size_t)3 * n, kBlock)),
                dim3(kBlock), n, pos, vel, (const float*)ctx->F.ptr, kick, dt,
                per_atom ? (const double*)ctx->masses.ptr : (const double*)nullptr,
                (const int*)ctx->sys.perm.ptr, mass);
  return hipGetLastError();
}

}  // namespace nep
