// Neighbour lists on gfx950.
//
// The site environment of atom i is every (j, lattice image n) with
// |r_j + n.H - r_i| < r_c (paper, Sec. II A), with r_c = r_c^R + skin.
// Entries closer than r_c^A + skin are stored first, so the angular loop of
// the descriptor kernel runs over a prefix of the radial list.
//
// Large boxes (at least three cells of width r_c along every cell vector):
// atoms are binned by fractional coordinate, each cell's members are sorted
// by index (so the list order does not depend on atomic arrival order) and
// each atom scans its 27 surrounding cells.  Thin boxes: every atom is tested
// against every atom and every image in a bounded range.
//
// The membership test is evaluated in float64 exactly as documented in
// nep.h (no fused multiply-add), so the list is reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "nep_device.h"

namespace nep {
namespace {

__device__ __forceinline__ void fractional(const Box& b, const double r[3], double s[3]) {
  for (int a = 0; a < 3; ++a) s[a] = r[0] * b.hinv[a] + r[1] * b.hinv[3 + a] + r[2] * b.hinv[6 + a];
}

__global__ void k_zero(int* __restrict__ a, int m) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) a[t] = 0;
}

// Integer cell offsets w = floor(s) of every atom (optionally wrapping the
// positions into the cell first) and, on the cell path, the cell index.
__global__ void k_bin(int n, double* __restrict__ pos, Box box, int nc0, int nc1, int nc2,
                      int use_cells, int wrap_in_place, int* __restrict__ wrap,
                      int* __restrict__ cell_of, int* __restrict__ cell_cnt,
                      float* __restrict__ pos_ref) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double r[3] = {pos[i], pos[n + i], pos[2 * n + i]};
  double s[3];
  int w[3];
  fractional(box, r, s);
  for (int a = 0; a < 3; ++a) w[a] = (int)floor(s[a]);
  if (wrap_in_place && (w[0] | w[1] | w[2])) {
    for (int c = 0; c < 3; ++c) {
      r[c] -= ((double)w[0] * box.h[c] + (double)w[1] * box.h[3 + c]) + (double)w[2] * box.h[6 + c];
      pos[c * n + i] = r[c];
    }
    fractional(box, r, s);
    for (int a = 0; a < 3; ++a) w[a] = (int)floor(s[a]);
  }
  for (int a = 0; a < 3; ++a) wrap[a * n + i] = w[a];
  if (pos_ref)  // the positions this list is built for (no re-sort on this path)
    for (int c = 0; c < 3; ++c) pos_ref[c * n + i] = (float)r[c];
  if (use_cells) {
    const int nc[3] = {nc0, nc1, nc2};
    int c[3];
    for (int a = 0; a < 3; ++a) {
      int ca = (int)((s[a] - (double)w[a]) * (double)nc[a]);
      c[a] = ca < 0 ? 0 : (ca >= nc[a] ? nc[a] - 1 : ca);
    }
    int cell = (c[2] * nc1 + c[1]) * nc0 + c[0];
    cell_of[i] = cell;
    atomicAdd(&cell_cnt[cell], 1);
  }
}

// Exclusive prefix sum of m <= 1024 * kScanChunks counts by one block of
// 1024 threads; the counts are cleared for the next build and the fill
// counters for k_fill.
constexpr int kScanChunks = 16;
__global__ __launch_bounds__(1024) void k_scan(int m, int* __restrict__ cnt,
                                               int* __restrict__ start, int* __restrict__ fill) {
  // wave w owns a run of `chunks` chunks of 64 consecutive cells (coalesced
  // reads, all issued before any is used); each chunk is scanned across the
  // lanes, the chunks of a wave in order, the 16 waves after one barrier
  __shared__ int wsum[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int chunks = (m + 1023) / 1024;
  const int c0 = w * chunks * 64;
  int own[kScanChunks], x[kScanChunks];
#pragma unroll
  for (int t = 0; t < kScanChunks; ++t) {
    const int c = c0 + 64 * t + lane;
    own[t] = t < chunks && c < m ? cnt[c] : 0;
    x[t] = own[t];
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1)
#pragma unroll
    for (int t = 0; t < kScanChunks; ++t)
      if (t < chunks) {
        const int y = __shfl_up(x[t], d, 64);
        if (lane >= d) x[t] += y;
      }
  int run = 0;  // the wave's sum before chunk t
  int before[kScanChunks];
#pragma unroll
  for (int t = 0; t < kScanChunks; ++t) {
    before[t] = run;
    if (t < chunks) run += __shfl(x[t], 63, 64);
  }
  if (lane == 0) wsum[w] = run;
  __syncthreads();
  int carry = 0;
  for (int u = 0; u < w; ++u) carry += wsum[u];
#pragma unroll
  for (int t = 0; t < kScanChunks; ++t) {
    const int c = c0 + 64 * t + lane;
    if (t < chunks && c < m) {
      start[c] = carry + before[t] + x[t] - own[t];
      cnt[c] = 0;   // ready for the next build
      fill[c] = 0;  // for k_fill, next
    }
  }
  if (threadIdx.x == 1023) {
    int tot = 0;
    for (int u = 0; u < 16; ++u) tot += wsum[u];
    start[m] = tot;
  }
}

// The same scan for many cells in three launches: block b scans counts
// [1024 b, 1024 b + 1024) (k_scan_blocks), one block scans the block totals
// (k_scan_totals), every block adds its offset and clears the counters
// (k_scan_add).
__device__ __forceinline__ int block_exclusive_scan_1024(int v, int* part, int& total) {
  const int t = threadIdx.x;
  part[t] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int u = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += u;
    __syncthreads();
  }
  total = part[1023];
  return part[t] - v;
}

__global__ __launch_bounds__(1024) void k_scan_blocks(int m, const int* __restrict__ cnt,
                                                      int* __restrict__ start,
                                                      int* __restrict__ block_total) {
  __shared__ int part[1024];
  const int k = blockIdx.x * 1024 + threadIdx.x;
  int total;
  const int ex = block_exclusive_scan_1024(k < m ? cnt[k] : 0, part, total);
  if (k < m) start[k] = ex;
  if (threadIdx.x == 0) block_total[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_totals(int nb, int m, int* __restrict__ block_total,
                                                      int* __restrict__ start) {
  __shared__ int part[1024];
  int total;
  const int v = threadIdx.x < nb ? block_total[threadIdx.x] : 0;
  const int ex = block_exclusive_scan_1024(v, part, total);
  __syncthreads();
  if (threadIdx.x < nb) block_total[threadIdx.x] = ex;
  if (threadIdx.x == 0) start[m] = total;
}

__global__ void k_scan_add(int m, const int* __restrict__ block_offset, int* __restrict__ start,
                           int* __restrict__ cnt, int* __restrict__ fill) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  start[k] += block_offset[k / 1024];
  cnt[k] = 0;   // ready for the next build
  fill[k] = 0;  // for k_fill, next
}

__global__ void k_fill(int n, const int* __restrict__ cell_of, const int* __restrict__ start,
                       int* __restrict__ fill, int* __restrict__ members) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = cell_of[i];
  int slot = atomicAdd(&fill[c], 1);
  members[start[c] + slot] = i;
}

// Order every cell's members by atom index: each atom counts the members of
// its cell with a smaller index and takes that place (cells are small).
// Re-sort atoms into cell order (cells in order, each cell's members by old
// index): old atom o finds its rank among its cell's members and moves to
// internal index k = start[cell] + rank.  Position, velocity (when given),
// offsets, caller index and cell move with it, and a 32-byte record
// (position, index, packed offsets) is written per atom.
__global__ void k_rank_permute(int n, const int* __restrict__ start,
                               const int* __restrict__ members, const double* __restrict__ pos,
                               double* __restrict__ pos_out, const double* __restrict__ vel,
                               double* __restrict__ vel_out, const int* __restrict__ wrap,
                               int* __restrict__ wrap_out, const int* __restrict__ perm,
                               int* __restrict__ perm_out, const int* __restrict__ cell_of,
                               int* __restrict__ cell_out, CellRec* __restrict__ rec,
                               int* __restrict__ iperm_out, float* __restrict__ pos_ref,
                               int* __restrict__ flags) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const int c = cell_of[o];
  const int b = start[c], e = start[c + 1];
  int rank = 0;
  for (int m = b; m < e; ++m) rank += members[m] < o ? 1 : 0;
  const int k = b + rank;
  CellRec r;
  r.x = pos[o];
  r.y = pos[n + o];
  r.z = pos[2 * n + o];
  pos_out[k] = r.x;
  pos_out[n + k] = r.y;
  pos_out[2 * n + k] = r.z;
  pos_ref[k] = (float)r.x;
  pos_ref[n + k] = (float)r.y;
  pos_ref[2 * n + k] = (float)r.z;
  if (vel) {
    vel_out[k] = vel[o];
    vel_out[n + k] = vel[n + o];
    vel_out[2 * n + k] = vel[2 * n + o];
  }
  const int w0 = wrap[o], w1 = wrap[n + o], w2 = wrap[2 * n + o];
  wrap_out[k] = w0;
  wrap_out[n + k] = w1;
  wrap_out[2 * n + k] = w2;
  const int caller = perm[o];
  perm_out[k] = caller;
  iperm_out[caller] = k;  // caller index -> new internal index
  cell_out[k] = c;
  if (w0 < -127 || w0 > 127 || w1 < -127 || w1 > 127 || w2 < -127 || w2 > 127)
    flags[kFlagImage] = 1;
  r.j = k;
  r.w = (w0 & 0xFF) | ((w1 & 0xFF) << 8) | ((w2 & 0xFF) << 16);
  rec[k] = r;
}

template <class T>
__global__ void k_take_rows(int n, int rows, const T* __restrict__ src, const int* __restrict__ perm,
                            T* __restrict__ dst) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int o = perm[k];
  for (int r = 0; r < rows; ++r) dst[(size_t)r * n + k] = src[(size_t)r * n + o];
}

template <class T>
__global__ void k_put_rows(int n, int rows, const T* __restrict__ src, const int* __restrict__ iperm,
                           T* __restrict__ dst) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int k = iperm[c];
  for (int r = 0; r < rows; ++r) dst[(size_t)r * n + c] = src[(size_t)r * n + k];
}

// Two [3][n] arrays back to the caller's order in one pass.
__global__ void k_put_rows2(int n, const double* __restrict__ a, double* __restrict__ a_dst,
                            const double* __restrict__ b, double* __restrict__ b_dst,
                            const int* __restrict__ iperm) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int k = iperm[c];
  for (int r = 0; r < 3; ++r) {
    a_dst[(size_t)r * n + c] = a[(size_t)r * n + k];
    b_dst[(size_t)r * n + c] = b[(size_t)r * n + k];
  }
}

// iperm[perm[k]] = k.
__global__ void k_invert_perm(int n, const int* __restrict__ perm, int* __restrict__ iperm) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) iperm[perm[k]] = k;
}

__global__ void k_iota(int n, int* __restrict__ a) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) a[k] = k;
}

// One block per cell: the records of the 27 surrounding cells are staged in
// LDS once (up to MAXC of them; the rest are read from global memory) and
// every atom of the cell is scanned by a group of G lanes.  The candidates are
// numbered consecutively (cell order, then member order) and the G lanes test
// G consecutive candidates at a time; a ballot and a population count give
// each kept entry the slot a serial scan would give it, so the order does not
// depend on G.  Angular-range entries go to the list at once; the remaining
// radial-range entries wait in LDS (up to RO per atom) and follow them when
// the scan is done.  An atom with more than RO of them scans its cells a
// second time for that part.  When all candidates fit in LDS (MAXC), LDS
// holds each one's position relative to the cell centre in float32, a
// float32 first pass picks the candidates that can be inside the larger
// cutoff (up to SC of them, their numbers in scan order in LDS) and the exact
// test runs on those alone, with their float64 records read from global
// memory; the lists are the same as those of the plain scan.  Atoms are in
// cell order, so a cell's atoms are start[c] .. start[c+1]-1.
template <int G, int RO, int SC, int MAXC, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8))) void k_build_cells(
    int n, int cap, const double* __restrict__ pos, Box box, int nc0, int nc1, int nc2,
    const int* __restrict__ wrap, const int* __restrict__ start,
    const CellRec* __restrict__ rec, double rc2_r, double rc2_a, uint32_t* __restrict__ nl,
    uint32_t* __restrict__ nl_rm, int* __restrict__ cnt_r, int* __restrict__ cnt_a,
    int* __restrict__ flags) {
  static_assert(G == 32 || G == 64, "lane groups inside one wave");
  constexpr int NG = NT / G;  // atoms scanned side by side
  __shared__ int s_off[28];    // first candidate number of each neighbour cell
  __shared__ int s_first[27];  // first member slot of each neighbour cell
  __shared__ int s_img[27];    // packed periodic image offset of each neighbour cell
  __shared__ double s_shift[27][3];  // its lattice shift (for atoms with equal offsets)
  __shared__ float4 s_pf[MAXC];  // candidate position - cell centre (float32), wrap offsets
  __shared__ uint8_t s_cell[MAXC];
  __shared__ uint32_t s_ro[NG][RO];  // radial-only entries in scan order
  __shared__ uint16_t s_cand[NG][SC];  // candidates left by the first pass
  static_assert(MAXC <= 65536, "candidate numbers in 16 bits");
  const int cell = (int)xcd_block(blockIdx.x, gridDim.x);
  const int c0 = cell % nc0, c1 = (cell / nc0) % nc1, c2 = cell / (nc0 * nc1);
  const int tid = threadIdx.x;
  // thread q < 27 looks up neighbour cell q (offsets o2, o1, o0 in -1..1, o0 fastest)
  if (tid < 27) {
    const int e0 = c0 + tid % 3 - 1, e1 = c1 + (tid / 3) % 3 - 1, e2 = c2 + tid / 9 - 1;
    const int m0 = e0 < 0 ? -1 : (e0 >= nc0 ? 1 : 0);
    const int m1 = e1 < 0 ? -1 : (e1 >= nc1 ? 1 : 0);
    const int m2 = e2 < 0 ? -1 : (e2 >= nc2 ? 1 : 0);
    const int cc = ((e2 - m2 * nc2) * nc1 + (e1 - m1 * nc1)) * nc0 + (e0 - m0 * nc0);
    const int b = start[cc];
    s_first[tid] = b;
    s_off[tid + 1] = start[cc + 1] - b;
    s_img[tid] = (m0 + 1) | ((m1 + 1) << 2) | ((m2 + 1) << 4);
    image_shift(m0, m1, m2, box.h, s_shift[tid][0], s_shift[tid][1], s_shift[tid][2]);
  }
  __syncthreads();
  if (tid == 0) {
    s_off[0] = 0;
    for (int q = 1; q <= 27; ++q) s_off[q] += s_off[q - 1];
  }
  __syncthreads();
  const int total = s_off[27];
  if (tid < 27)
    for (int c = s_off[tid]; c < s_off[tid + 1] && c < MAXC; ++c) s_cell[c] = (uint8_t)tid;
  __syncthreads();
  // the cell centre: the first pass works on coordinates relative to it
  const double f0 = (c0 + 0.5) / nc0, f1 = (c1 + 0.5) / nc1, f2 = (c2 + 0.5) / nc2;
  const double ox = f0 * box.h[0] + f1 * box.h[3] + f2 * box.h[6];
  const double oy = f0 * box.h[1] + f1 * box.h[4] + f2 * box.h[7];
  const double oz = f0 * box.h[2] + f1 * box.h[5] + f2 * box.h[8];
  if (total <= MAXC)
    for (int c = tid; c < total; c += NT) {
      const int q = s_cell[c];
      const CellRec r = rec[s_first[q] + (c - s_off[q])];
      s_pf[c] = make_float4((float)((r.x + s_shift[q][0]) - ox), (float)((r.y + s_shift[q][1]) - oy),
                            (float)((r.z + s_shift[q][2]) - oz), __int_as_float(r.w & 0xFFFFFF));
    }
  __syncthreads();

  const int grp = tid / G;
  const int k = tid % G;
  const int shift = (tid & 63) - k;  // first lane of the group within its wave
  const unsigned long long below = (1ull << k) - 1ull;
  const unsigned long long gmask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
  const int a1 = start[cell + 1];
  // First-pass bound.  For an atom within kNear of the cell centre (each
  // component) and a candidate with its wrap offsets whose true displacement
  // d has |d| < r_c (the larger cutoff), each float32 displacement component
  // is off by at most eps = 2^-22 (kNear + r_c) (three roundings of values
  // below kNear + r_c), so |d_f| < r_c + 2 eps and the float32 |d_f|^2 (three
  // roundings) stays below thr: such a candidate always passes.
  constexpr float kNear = 4096.f;
  const double rcm = sqrt(fmax(rc2_r, rc2_a));
  const double eps = 0x1p-22 * ((double)kNear + rcm);
  const float thr = (float)((rcm + 2.0 * eps) * (rcm + 2.0 * eps) * (1.0 + 0x1p-20));
  // records from LDS when all candidates were staged, else all from global
  // memory (two instantiations, so that neither path uses generic addresses)
  auto scan = [&](auto staged) {
  for (int i = start[cell] + grp; i < a1; i += NG) {
    const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
    const int wi0 = wrap[i], wi1 = wrap[n + i], wi2 = wrap[2 * n + i];
    bool overflow = false, bad_image = false;
    // candidate c: its list entry and squared distance (r2 < 0 for the atom itself)
    auto candidate = [&](int c, uint32_t& entry, double& r2) {
      int q;  // the cell that holds candidate c: off[q] <= c < off[q+1]
      CellRec rc;
      if constexpr (decltype(staged)::value) {
        q = s_cell[c];
        rc = rec[s_first[q] + (c - s_off[q])];
      } else {
        int lo = 0, hi = 27;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_off[mid] <= c)
            lo = mid;
          else
            hi = mid;
        }
        q = lo;
        rc = rec[s_first[q] + (c - s_off[q])];
      }
      const int im = s_img[q];
      const int j = rc.j;
      const int d0 = wi0 - (int)(signed char)(rc.w & 0xFF);
      const int d1 = wi1 - (int)(signed char)((rc.w >> 8) & 0xFF);
      const int d2 = wi2 - (int)(signed char)((rc.w >> 16) & 0xFF);
      const int n0 = (im & 3) - 1 + d0;
      const int n1 = ((im >> 2) & 3) - 1 + d1;
      const int n2 = ((im >> 4) & 3) - 1 + d2;
      r2 = -1.0;
      entry = 0;
      if (!(j == i && n0 == 0 && n1 == 0 && n2 == 0)) {
        if ((d0 | d1 | d2) == 0)  // the neighbour cell's own shift (atoms in the cell)
          r2 = list_r2_shifted(rc.x, rc.y, rc.z, xi, yi, zi, s_shift[q][0], s_shift[q][1],
                               s_shift[q][2]);
        else
          r2 = list_r2(rc.x, rc.y, rc.z, xi, yi, zi, n0, n1, n2, box.h);
        if (r2 < rc2_r && (n0 < -3 || n0 > 3 || n1 < -3 || n1 > 3 || n2 < -3 || n2 > 3)) {
          bad_image = true;
          r2 = -1.0;
        }
        entry = pack_entry(j, n0, n1, n2);
      }
    };
    // First pass over the staged positions.  A candidate with the atom's own
    // wrap counts (d = 0 below) is left out only if its float32 distance
    // exceeds the bound thr above; every other candidate (and every
    // candidate of an atom beyond kNear of the cell centre) is left to the
    // exact test.  So the exact test sees every candidate it would keep, in
    // scan order.
    int ncand = total;
    bool listed = false;
    if constexpr (decltype(staged)::value) {
      const bool in_range = wi0 >= -128 && wi0 <= 127 && wi1 >= -128 && wi1 <= 127 &&
                            wi2 >= -128 && wi2 <= 127;
      const float xf = (float)(xi - ox), yf = (float)(yi - oy), zf = (float)(zi - oz);
      const bool near = fabsf(xf) <= kNear && fabsf(yf) <= kNear && fabsf(zf) <= kNear;
      const int wpack = in_range && near
                            ? (wi0 & 0xFF) | ((wi1 & 0xFF) << 8) | ((wi2 & 0xFF) << 16)
                            : -1;
      int nk = 0;
      for (int base = 0; base < total; base += G) {
        const int c = base + k;
        bool pass = false;
        if (c < total) {
          const float4 pf = s_pf[c];
          const float ex = pf.x - xf, ey = pf.y - yf, ez = pf.z - zf;
          const float r2f = __builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, ex * ex));
          pass = __float_as_int(pf.w) != wpack || r2f < thr;
        }
        const unsigned long long bp = (__ballot(pass) >> shift) & gmask;
        if (pass) {
          const int u = nk + __popcll(bp & below);
          if (u < SC) s_cand[grp][u] = (uint16_t)c;
        }
        nk += __popcll(bp);
      }
      if (nk <= SC) {
        ncand = nk;
        listed = true;
      }
      // the list is read back by other lanes of the group below
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // the t-th candidate of the exact test
    auto number = [&](int t) { return listed ? (int)s_cand[grp][t] : t; };
    int na = 0, nro = 0;
    for (int base = 0; base < ncand; base += G) {
      const int t = base + k;
      bool keep_a = false, keep_r = false;
      uint32_t entry = 0;
      if (t < ncand) {
        double r2;
        candidate(number(t), entry, r2);
        keep_a = r2 >= 0.0 && r2 < rc2_a;
        keep_r = r2 >= rc2_a && r2 < rc2_r;
      }
      const unsigned long long ba = (__ballot(keep_a) >> shift) & gmask;
      const unsigned long long br = (__ballot(keep_r) >> shift) & gmask;
      if (keep_a) {
        const int slot = na + __popcll(ba & below);
        if (slot < cap) {
          nl[(size_t)slot * n + i] = entry;
          nl_rm[(size_t)i * cap + slot] = entry;
        } else {
          overflow = true;
        }
      }
      if (keep_r) {
        const int ro = nro + __popcll(br & below);
        if (ro < RO) s_ro[grp][ro] = entry;
      }
      na += __popcll(ba);
      nro += __popcll(br);
    }
    if (nro <= RO) {
      // the group's LDS writes above are read back by other lanes of the group
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int t = k; t < nro; t += G) {
        const int slot = na + t;
        if (slot < cap) {
          nl[(size_t)slot * n + i] = s_ro[grp][t];
          nl_rm[(size_t)i * cap + slot] = s_ro[grp][t];
        } else {
          overflow = true;
        }
      }
    } else {
      int count = na;
      for (int base = 0; base < ncand; base += G) {
        const int t = base + k;
        bool keep = false;
        uint32_t entry = 0;
        if (t < ncand) {
          double r2;
          candidate(number(t), entry, r2);
          keep = r2 >= rc2_a && r2 < rc2_r;
        }
        const unsigned long long ball = (__ballot(keep) >> shift) & gmask;
        if (keep) {
          const int slot = count + __popcll(ball & below);
          if (slot < cap) {
            nl[(size_t)slot * n + i] = entry;
            nl_rm[(size_t)i * cap + slot] = entry;
          } else {
            overflow = true;
          }
        }
        count += __popcll(ball);
      }
    }
    if (k == 0) {
      cnt_a[i] = min(na, cap);
      cnt_r[i] = min(na + nro, cap);
    }
    if (overflow) flags[kFlagOverflow] = 1;
    if (bad_image) flags[kFlagImage] = 1;
    // the group reuses s_ro for its next atom
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  };
  if (total <= MAXC)
    scan(std::true_type{});
  else
    scan(std::false_type{});
}

// One 64-lane wave per atom (4 atoms per block): every atom j and every image
// m in [-k, k]^3 of the wrapped frame (boxes thinner than three cut-off
// widths).  Candidate c = j (2k+1)^3 + image (m2 fastest) is tested by lane
// c mod 64; a ballot and a population count give each kept entry the slot of
// the serial order (angular-range entries first, then the radial-only ones).
__global__ __launch_bounds__(256) void k_build_all_pairs(
    int n, int cap, const double* __restrict__ pos, Box box, int k0, int k1, int k2,
    const int* __restrict__ wrap, double rc2_r, double rc2_a, uint32_t* __restrict__ nl,
    int* __restrict__ cnt_r, int* __restrict__ cnt_a, int* __restrict__ flags) {
  const int lane = (int)threadIdx.x % 64;
  const int i = (int)blockIdx.x * 4 + (int)threadIdx.x / 64;
  if (i >= n) return;  // whole waves leave together
  const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
  const int wi0 = wrap[i], wi1 = wrap[n + i], wi2 = wrap[2 * n + i];
  const int d1 = 2 * k1 + 1, d2 = 2 * k2 + 1;
  const int nimg = (2 * k0 + 1) * d1 * d2;
  const long long total = (long long)n * nimg;
  const unsigned long long below = (1ull << lane) - 1ull;
  int count = 0;
  bool overflow = false, bad_image = false;
  for (int pass = 0; pass < 2; ++pass) {
    for (long long base = 0; base < total; base += 64) {
      const long long c = base + lane;
      bool keep = false;
      uint32_t entry = 0;
      if (c < total) {
        const int j = (int)(c / nimg), im = (int)(c % nimg);
        const int m0 = im / (d1 * d2) - k0, m1 = (im / d2) % d1 - k1, m2 = im % d2 - k2;
        const int n0 = m0 + wi0 - wrap[j], n1 = m1 + wi1 - wrap[n + j], n2 = m2 + wi2 - wrap[2 * n + j];
        if (!(j == i && n0 == 0 && n1 == 0 && n2 == 0)) {
          const double r2 = list_r2(pos[j], pos[n + j], pos[2 * n + j], xi, yi, zi, n0, n1, n2, box.h);
          const bool in_a = r2 < rc2_a;
          keep = pass == 0 ? in_a : (!in_a && r2 < rc2_r);
          if (keep && (n0 < -3 || n0 > 3 || n1 < -3 || n1 > 3 || n2 < -3 || n2 > 3)) {
            bad_image = true;
            keep = false;
          }
          entry = pack_entry(j, n0, n1, n2);
        }
      }
      const unsigned long long b = __ballot(keep);
      if (keep) {
        const int slot = count + __popcll(b & below);
        if (slot < cap)
          nl[(size_t)slot * n + i] = entry;
        else
          overflow = true;
      }
      count += __popcll(b);
    }
    if (pass == 0 && lane == 0) cnt_a[i] = min(count, cap);
  }
  if (lane == 0) cnt_r[i] = min(count, cap);
  if (overflow) flags[kFlagOverflow] = 1;
  if (bad_image) flags[kFlagImage] = 1;
}

// Slot of the reverse entry (i, -n) in atom j's list, for every entry (j, n)
// of atom i.  One thread per (slot, atom).  |r_ji| = |r_ij| exactly, so the
// reverse entry lies in the same part (angular prefix or radial rest) of j's
// list and only that part is searched.  The lists are symmetric unless a list
// was cut at its capacity (the overflow flag), so the thread of an entry with
// j > i also writes the reverse slot of the entry it finds, and entries with
// j < i are left to that thread; after an overflow every entry searches for
// itself, so that every reverse slot still names a slot inside j's list.
// One block per kReverseAtoms consecutive atoms (all their slots), blocks
// spread over the XCDs in contiguous ranges: a pair's partner row is then
// mostly a nearby atom's, already in the XCD's L2.
constexpr int kReverseAtoms = 32;
__global__ __launch_bounds__(kBlock) void k_reverse(int n, int cap, const uint32_t* __restrict__ nl,
                          const uint32_t* __restrict__ nl_rm, const int* __restrict__ cnt_r,
                          const int* __restrict__ cnt_a, int* __restrict__ rev,
                          int* __restrict__ flags) {
  // thread (s0, i) handles slots s0, s0 + width, ... of atom i
  constexpr int width = kBlock / kReverseAtoms;
  const int i = (int)xcd_block(blockIdx.x, gridDim.x) * kReverseAtoms + threadIdx.x % kReverseAtoms;
  if (i >= n) return;
  const int cr = cnt_r[i], ca = cnt_a[i];
  const bool symmetric = flags[kFlagOverflow] == 0;
  // kBatch slots of the thread at a time: their entries, then their
  // partners' list counts, are read before the first search
  constexpr int kBatch = 4;
  for (int sb = threadIdx.x / kReverseAtoms; sb < cr; sb += width * kBatch) {
    uint32_t eb[kBatch];
    int pa[kBatch], pr[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int s = sb + b * width;
      eb[b] = s < cr ? nl[(size_t)s * n + i] : 0u;
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int s = sb + b * width;
      const int j = (int)(eb[b] & kAtomMask);
      const bool need = s < cr && !(symmetric && j < i);
      pa[b] = need ? cnt_a[j] : 0;
      pr[b] = need ? cnt_r[j] : 0;
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int s = sb + b * width;
      if (s >= cr) break;
      const size_t idx = (size_t)s * n + i;
      const uint32_t e = eb[b];
      const int j = (int)(e & kAtomMask);
      if (symmetric && j < i) continue;
      int n0, n1, n2;
      unpack_image(e, n0, n1, n2);
      const uint32_t target = pack_entry(i, -n0, -n1, -n2);
      const bool angular = s < ca;
      const int t0 = angular ? 0 : pa[b];
      const int t1 = angular ? pa[b] : pr[b];
      int found = -1;
      if (nl_rm && (cap & 3) == 0) {  // j's entries are contiguous: 4 per load
        // 16 entries per round, their four loads issued together (no load
        // waits on the previous compare); loads stay below t1 <= cap
        const uint4* row4 = reinterpret_cast<const uint4*>(nl_rm + (size_t)j * cap);
        for (int u16 = t0 & ~3; u16 < t1 && found < 0; u16 += 16) {
          uint4 v[4];
#pragma unroll
          for (int q = 0; q < 4; ++q)
            v[q] = u16 + 4 * q < t1 ? row4[(u16 >> 2) + q] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int u4 = u16 + 4 * q;
            if (found >= 0 || u4 >= t1) continue;
            if (v[q].x == target && u4 >= t0) found = u4;
            else if (v[q].y == target && u4 + 1 >= t0 && u4 + 1 < t1) found = u4 + 1;
            else if (v[q].z == target && u4 + 2 >= t0 && u4 + 2 < t1) found = u4 + 2;
            else if (v[q].w == target && u4 + 3 >= t0 && u4 + 3 < t1) found = u4 + 3;
          }
        }
      } else if (nl_rm) {
        const uint32_t* row = nl_rm + (size_t)j * cap;
        for (int u = t0; u < t1; ++u) {
          if (row[u] == target) {
            found = u;
            break;
          }
        }
      } else {
        for (int u = t0; u < t1; ++u) {
          if (nl[(size_t)u * n + j] == target) {
            found = u;
            break;
          }
        }
      }
      if (found < 0) {
        flags[kFlagReverse] = 1;
        found = 0;
      } else if (symmetric && j != i) {
        rev[(size_t)found * n + j] = s;
      }
      rev[idx] = found;
    }
  }
}

// Expand the list into the caller's atom numbering: slot s of caller atom
// perm[k] holds caller atom perm[j].
__global__ void k_unpack(int n, int cap, const uint32_t* __restrict__ nl,
                         const int* __restrict__ perm, const int* __restrict__ cnt_r,
                         const int* __restrict__ cnt_a, const int* __restrict__ rev,
                         int* __restrict__ nbr, int* __restrict__ img, int* __restrict__ cnt_r_out,
                         int* __restrict__ cnt_a_out, int* __restrict__ rev_out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * cap) return;
  const int k = (int)(idx % (size_t)n);
  const int s = (int)(idx / (size_t)n);
  const size_t out = (size_t)s * n + perm[k];
  if (s == 0) {
    if (cnt_r_out) cnt_r_out[perm[k]] = cnt_r[k];
    if (cnt_a_out) cnt_a_out[perm[k]] = cnt_a[k];
  }
  if (s >= cnt_r[k]) return;
  const uint32_t e = nl[idx];
  int n0, n1, n2;
  unpack_image(e, n0, n1, n2);
  if (nbr) nbr[out] = perm[(int)(e & kAtomMask)];
  if (img) {
    img[3 * out] = n0;
    img[3 * out + 1] = n1;
    img[3 * out + 2] = n2;
  }
  if (rev_out) rev_out[out] = rev[idx];
}

inline unsigned blocks_for(size_t work, int block) { return (unsigned)((work + block - 1) / block); }

}  // namespace

void launch_reverse(nep_ctx ctx, int n, int cap, const uint32_t* nl, const int* cnt_r,
                    const int* cnt_a, int* rev) {
  const size_t ncap = (size_t)n * cap;
  if (ncap == 0) return;
  launch_kernel(ctx, false, false, k_reverse, dim3(blocks_for((size_t)n, kReverseAtoms)),
                dim3(kBlock), n, cap, nl, (const uint32_t*)nullptr, cnt_r, cnt_a, rev,
                ctx->flags.ptr);
}

hipError_t unpack_neighbors(nep_ctx ctx, int* nbr, int* img, int* cnt_r, int* cnt_a, int* rev) {
  const System& s = ctx->sys;
  const size_t ncap = (size_t)s.n * s.cap;
  if (ncap == 0) return hipSuccess;
  k_unpack<<<blocks_for(ncap, kBlock), kBlock, 0, ctx->stream>>>(
      s.n, s.cap, s.nl.ptr, s.perm.ptr, s.cnt_r.ptr, s.cnt_a.ptr, s.rev.ptr, nbr, img, cnt_r,
      cnt_a, rev);
  return hipGetLastError();
}

void launch_take_rows(nep_ctx ctx, int n, int rows, const double* src, double* dst) {
  if (n == 0) return;
  launch_kernel(ctx, false, false, k_take_rows<double>, dim3(blocks_for(n, kBlock)), dim3(kBlock),
                n, rows, src, (const int*)ctx->sys.perm.ptr, dst);
}

void launch_put_rows(nep_ctx ctx, int n, int rows, const double* src, double* dst) {
  if (n == 0) return;
  launch_kernel(ctx, false, false, k_put_rows<double>, dim3(blocks_for(n, kBlock)), dim3(kBlock),
                n, rows, src, (const int*)ctx->sys.iperm.ptr, dst);
}

void launch_put_rows2(nep_ctx ctx, int n, const double* a, double* a_dst, const double* b,
                      double* b_dst) {
  if (n == 0) return;
  launch_kernel(ctx, false, false, k_put_rows2, dim3(blocks_for(n, kBlock)), dim3(kBlock), n, a,
                a_dst, b, b_dst, (const int*)ctx->sys.iperm.ptr);
}

void launch_put_rows(nep_ctx ctx, int n, int rows, const float* src, float* dst) {
  if (n == 0) return;
  launch_kernel(ctx, false, false, k_put_rows<float>, dim3(blocks_for(n, kBlock)), dim3(kBlock), n,
                rows, src, (const int*)ctx->sys.iperm.ptr, dst);
}

void launch_iota(nep_ctx ctx, int n, int* dst) {
  if (n == 0) return;
  launch_kernel(ctx, false, false, k_iota, dim3(blocks_for(n, kBlock)), dim3(kBlock), n, dst);
}

void prepare_system_geometry(System& s, const double* H, double rc_r, double rc_a, double skin) {
  for (int k = 0; k < 9; ++k) s.box.h[k] = H[k];
  const double a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7],
               k = H[8];
  const double det = a * (e * k - f * h) - b * (d * k - f * g) + c * (d * h - e * g);
  double* hi = s.box.hinv;
  hi[0] = (e * k - f * h) / det;
  hi[1] = (c * h - b * k) / det;
  hi[2] = (b * f - c * e) / det;
  hi[3] = (f * g - d * k) / det;
  hi[4] = (a * k - c * g) / det;
  hi[5] = (c * d - a * f) / det;
  hi[6] = (d * h - e * g) / det;
  hi[7] = (b * g - a * h) / det;
  hi[8] = (a * e - b * d) / det;
  s.skin = skin;
  s.rc_list_r = rc_r + skin;
  s.rc_list_a = rc_a + skin;
  const double vol = std::fabs(det);
  const double* A = H;
  const double* B = H + 3;
  const double* C = H + 6;
  auto cross_norm = [](const double* u, const double* v) {
    double x = u[1] * v[2] - u[2] * v[1], y = u[2] * v[0] - u[0] * v[2], z = u[0] * v[1] - u[1] * v[0];
    return std::sqrt(x * x + y * y + z * z);
  };
  const double width[3] = {vol / cross_norm(B, C), vol / cross_norm(C, A), vol / cross_norm(A, B)};
  s.use_cells = true;
  for (int ax = 0; ax < 3; ++ax) {
    s.nc[ax] = (int)std::floor(width[ax] / (s.rc_list_r * (1.0 + 1e-9)));
    if (s.nc[ax] < 3) s.use_cells = false;
    // wrapped fractional differences lie in (-1, 1); a neighbour needs
    // |ds + m| <= rc/width
    s.kimg[ax] = (int)std::floor(1.0 + s.rc_list_r / width[ax] * (1.0 + 1e-12) + 1e-12);
  }
  if (!s.use_cells) s.nc[0] = s.nc[1] = s.nc[2] = 1;
}

nep_status build_neighbors(nep_ctx ctx, bool wrap_in_place, bool have_vel) {
  System& s = ctx->sys;
  const int n = s.n;
  hipError_t e = hipSuccess;
  const size_t ncap = (size_t)n * s.cap;
  if ((e = s.nl.ensure(ncap)) != hipSuccess || (e = s.rev.ensure(ncap)) != hipSuccess ||
      (e = s.cnt_r.ensure(n)) != hipSuccess || (e = s.cnt_a.ensure(n)) != hipSuccess ||
      (e = s.iperm.ensure(n)) != hipSuccess || (e = s.pos_ref.ensure((size_t)3 * n)) != hipSuccess ||
      (e = s.wrap.ensure((size_t)3 * n)) != hipSuccess)
    return check_hip(ctx, e, "allocating neighbour lists");
  const double rc2_r = s.rc_list_r * s.rc_list_r;
  const double rc2_a = s.rc_list_a * s.rc_list_a;
  const dim3 blk(kBlock);
  if (s.use_cells) {
    const int ncell = s.nc[0] * s.nc[1] * s.nc[2];
    const int* cnt_before = s.cell_cnt.ptr;
    if ((e = s.nl_rm.ensure(ncap)) != hipSuccess || (e = s.cell_of.ensure(n)) != hipSuccess ||
        (e = s.cell_cnt.ensure(ncell)) != hipSuccess ||
        (e = s.scan_part.ensure(1024)) != hipSuccess ||
        (e = s.cell_start.ensure((size_t)ncell + 1)) != hipSuccess ||
        (e = s.cell_fill.ensure(ncell)) != hipSuccess ||
        (e = s.cell_atoms.ensure(n)) != hipSuccess ||
        (e = s.cell_rec.ensure(n)) != hipSuccess ||
        (e = s.pos_t.ensure((size_t)3 * n)) != hipSuccess ||
        (e = s.vel_t.ensure((size_t)3 * n)) != hipSuccess ||
        (e = s.perm_t.ensure(n)) != hipSuccess || (e = s.wrap_t.ensure((size_t)3 * n)) != hipSuccess ||
        (e = s.cell_t.ensure(n)) != hipSuccess)
      return check_hip(ctx, e, "allocating cell lists");
    const bool zero = s.cell_cnt.ptr != cnt_before || s.cells_zeroed_for != ncell;
    if (zero)
      launch_kernel(ctx, true, false, k_zero, dim3(blocks_for(ncell, kBlock)), blk,
                    s.cell_cnt.ptr, ncell);
    launch_kernel(ctx, !zero, false, k_bin, dim3(blocks_for(n, kBlock)), blk, n, s.pos_s.ptr,
                  s.box, s.nc[0], s.nc[1], s.nc[2], 1, wrap_in_place ? 1 : 0, s.wrap.ptr,
                  s.cell_of.ptr, s.cell_cnt.ptr, (float*)nullptr);
    const int nsb = (ncell + 1023) / 1024;
    if (ncell > 1024 * kScanChunks && nsb <= 1024) {
      launch_kernel(ctx, false, false, k_scan_blocks, dim3(nsb), dim3(1024), ncell,
                    (const int*)s.cell_cnt.ptr, s.cell_start.ptr, s.scan_part.ptr);
      launch_kernel(ctx, false, false, k_scan_totals, dim3(1), dim3(1024), nsb, ncell,
                    s.scan_part.ptr, s.cell_start.ptr);
      launch_kernel(ctx, false, false, k_scan_add, dim3(blocks_for(ncell, kBlock)), blk, ncell,
                    (const int*)s.scan_part.ptr, s.cell_start.ptr, s.cell_cnt.ptr,
                    s.cell_fill.ptr);
    } else {
      launch_kernel(ctx, false, false, k_scan, dim3(1), dim3(1024), ncell, s.cell_cnt.ptr,
                    s.cell_start.ptr, s.cell_fill.ptr);
    }
    s.cells_zeroed_for = ncell;
    launch_kernel(ctx, false, false, k_fill, dim3(blocks_for(n, kBlock)), blk, n,
                  (const int*)s.cell_of.ptr, (const int*)s.cell_start.ptr, s.cell_fill.ptr,
                  s.cell_atoms.ptr);
    launch_kernel(ctx, false, false, k_rank_permute, dim3(blocks_for(n, kBlock)), blk, n,
                  (const int*)s.cell_start.ptr, (const int*)s.cell_atoms.ptr,
                  (const double*)s.pos_s.ptr, s.pos_t.ptr,
                  have_vel ? (const double*)s.vel_s.ptr : (const double*)nullptr,
                  have_vel ? s.vel_t.ptr : (double*)nullptr, (const int*)s.wrap.ptr, s.wrap_t.ptr,
                  (const int*)s.perm.ptr, s.perm_t.ptr, (const int*)s.cell_of.ptr, s.cell_t.ptr,
                  s.cell_rec.ptr, s.iperm.ptr, s.pos_ref.ptr, ctx->flags.ptr);
    s.pos_s.swap(s.pos_t);
    if (have_vel) s.vel_s.swap(s.vel_t);
    s.wrap.swap(s.wrap_t);
    s.perm.swap(s.perm_t);
    s.cell_of.swap(s.cell_t);
    launch_kernel(ctx, false, false, k_build_cells<32, 64, 96, 640, 256>, dim3(ncell), dim3(256), n,
                  s.cap, (const double*)s.pos_s.ptr, s.box, s.nc[0], s.nc[1], s.nc[2],
                  (const int*)s.wrap.ptr, (const int*)s.cell_start.ptr,
                  (const CellRec*)s.cell_rec.ptr, rc2_r, rc2_a, s.nl.ptr, s.nl_rm.ptr, s.cnt_r.ptr,
                  s.cnt_a.ptr, ctx->flags.ptr);
  } else {
    launch_kernel(ctx, true, false, k_bin, dim3(blocks_for(n, kBlock)), blk, n, s.pos_s.ptr, s.box,
                  1, 1, 1, 0, wrap_in_place ? 1 : 0, s.wrap.ptr, (int*)nullptr, (int*)nullptr,
                  s.pos_ref.ptr);
    launch_kernel(ctx, false, false, k_build_all_pairs, dim3(blocks_for(n, 4)), dim3(256), n,
                  s.cap, (const double*)s.pos_s.ptr, s.box, s.kimg[0], s.kimg[1], s.kimg[2],
                  (const int*)s.wrap.ptr, rc2_r, rc2_a, s.nl.ptr, s.cnt_r.ptr, s.cnt_a.ptr,
                  ctx->flags.ptr);
  }
  // caller index -> internal index, for the coalesced copies back (the cell
  // path's k_rank_permute writes it)
  if (n > 0 && !s.use_cells)
    launch_kernel(ctx, false, false, k_invert_perm, dim3(blocks_for(n, kBlock)), blk, n,
                  (const int*)s.perm.ptr, s.iperm.ptr);
  launch_kernel(ctx, false, true, k_reverse, dim3(blocks_for((size_t)n, kReverseAtoms)), blk, n,
                s.cap, (const uint32_t*)s.nl.ptr,
                s.use_cells ? (const uint32_t*)s.nl_rm.ptr : (const uint32_t*)nullptr,
                (const int*)s.cnt_r.ptr, (const int*)s.cnt_a.ptr, s.rev.ptr, ctx->flags.ptr);
  return check_hip(ctx, hipGetLastError(), "launching neighbour kernels");
}

}  // namespace nep
