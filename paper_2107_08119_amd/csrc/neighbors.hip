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

#include "nep_internal.h"

namespace nep {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ void fractional(const Box& b, const double r[3], double s[3]) {
  for (int a = 0; a < 3; ++a) s[a] = r[0] * b.hinv[a] + r[1] * b.hinv[3 + a] + r[2] * b.hinv[6 + a];
}

// |r_j + n.H - r_i|^2 in the documented evaluation order.
__device__ __forceinline__ double pair_r2(const double* __restrict__ pos, int n, int j, double xi,
                                          double yi, double zi, int n0, int n1, int n2,
                                          const Box& b) {
#pragma clang fp contract(off)
  const double a0 = (double)n0, a1 = (double)n1, a2 = (double)n2;
  double dx = (pos[j] - xi) + ((a0 * b.h[0] + a1 * b.h[3]) + a2 * b.h[6]);
  double dy = (pos[n + j] - yi) + ((a0 * b.h[1] + a1 * b.h[4]) + a2 * b.h[7]);
  double dz = (pos[2 * n + j] - zi) + ((a0 * b.h[2] + a1 * b.h[5]) + a2 * b.h[8]);
  return (dx * dx + dy * dy) + dz * dz;
}

__global__ void k_zero(int* __restrict__ a, int m) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) a[t] = 0;
}

// Integer cell offsets w = floor(s) of every atom (optionally wrapping the
// positions into the cell first) and, on the cell path, the cell index.
__global__ void k_bin(int n, double* __restrict__ pos, Box box, int nc0, int nc1, int nc2,
                      int use_cells, int wrap_in_place, int* __restrict__ wrap,
                      int* __restrict__ cell_of, int* __restrict__ cell_cnt) {
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

// Exclusive prefix sum of m counts by one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan(int m, const int* __restrict__ cnt,
                                               int* __restrict__ start) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (m + 1023) / 1024;
  const int b = t * per;
  const int e = min(b + per, m);
  int sum = 0;
  for (int k = b; k < e; ++k) sum += cnt[k];
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = t > 0 ? part[t - 1] : 0;
  for (int k = b; k < e; ++k) {
    start[k] = run;
    run += cnt[k];
  }
  if (t == 1023) start[m] = part[1023];
}

__global__ void k_fill(int n, const int* __restrict__ cell_of, const int* __restrict__ start,
                       int* __restrict__ fill, int* __restrict__ members) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = cell_of[i];
  int slot = atomicAdd(&fill[c], 1);
  members[start[c] + slot] = i;
}

// Sort every cell's members by atom index (insertion sort; cells are small).
__global__ void k_sort_cells(int ncell, const int* __restrict__ start, int* __restrict__ members) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  int b = start[c], e = start[c + 1];
  for (int k = b + 1; k < e; ++k) {
    int v = members[k];
    int t = k - 1;
    while (t >= b && members[t] > v) {
      members[t + 1] = members[t];
      --t;
    }
    members[t + 1] = v;
  }
}

// One thread per atom: scan the 27 surrounding cells twice, first keeping the
// angular-range entries, then the remaining radial-range entries.
__global__ void k_build_cells(int n, int cap, const double* __restrict__ pos, Box box, int nc0,
                              int nc1, int nc2, const int* __restrict__ wrap,
                              const int* __restrict__ cell_of, const int* __restrict__ start,
                              const int* __restrict__ members, double rc2_r, double rc2_a,
                              uint32_t* __restrict__ nl, int* __restrict__ cnt_r,
                              int* __restrict__ cnt_a, int* __restrict__ flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
  const int wi0 = wrap[i], wi1 = wrap[n + i], wi2 = wrap[2 * n + i];
  const int cell = cell_of[i];
  const int c0 = cell % nc0, c1 = (cell / nc0) % nc1, c2 = cell / (nc0 * nc1);
  int count = 0;
  bool overflow = false, bad_image = false;
  for (int pass = 0; pass < 2; ++pass) {
    for (int o2 = -1; o2 <= 1; ++o2) {
      int d2 = c2 + o2;
      const int m2 = d2 < 0 ? -1 : (d2 >= nc2 ? 1 : 0);
      d2 -= m2 * nc2;
      for (int o1 = -1; o1 <= 1; ++o1) {
        int d1 = c1 + o1;
        const int m1 = d1 < 0 ? -1 : (d1 >= nc1 ? 1 : 0);
        d1 -= m1 * nc1;
        for (int o0 = -1; o0 <= 1; ++o0) {
          int d0 = c0 + o0;
          const int m0 = d0 < 0 ? -1 : (d0 >= nc0 ? 1 : 0);
          d0 -= m0 * nc0;
          const int cc = (d2 * nc1 + d1) * nc0 + d0;
          for (int t = start[cc]; t < start[cc + 1]; ++t) {
            const int j = members[t];
            const int n0 = m0 + wi0 - wrap[j];
            const int n1 = m1 + wi1 - wrap[n + j];
            const int n2 = m2 + wi2 - wrap[2 * n + j];
            if (j == i && n0 == 0 && n1 == 0 && n2 == 0) continue;
            const double r2 = pair_r2(pos, n, j, xi, yi, zi, n0, n1, n2, box);
            const bool in_a = r2 < rc2_a;
            const bool keep = pass == 0 ? in_a : (!in_a && r2 < rc2_r);
            if (!keep) continue;
            if (n0 < -3 || n0 > 3 || n1 < -3 || n1 > 3 || n2 < -3 || n2 > 3) {
              bad_image = true;
              continue;
            }
            if (count < cap)
              nl[(size_t)count * n + i] = pack_entry(j, n0, n1, n2);
            else
              overflow = true;
            ++count;
          }
        }
      }
    }
    if (pass == 0) cnt_a[i] = min(count, cap);
  }
  cnt_r[i] = min(count, cap);
  if (overflow) flags[kFlagOverflow] = 1;
  if (bad_image) flags[kFlagImage] = 1;
}

// One thread per atom: every atom j and every image m in [-k, k]^3 of the
// wrapped frame (boxes thinner than three cut-off widths).
__global__ void k_build_all_pairs(int n, int cap, const double* __restrict__ pos, Box box, int k0,
                                  int k1, int k2, const int* __restrict__ wrap, double rc2_r,
                                  double rc2_a, uint32_t* __restrict__ nl, int* __restrict__ cnt_r,
                                  int* __restrict__ cnt_a, int* __restrict__ flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
  const int wi0 = wrap[i], wi1 = wrap[n + i], wi2 = wrap[2 * n + i];
  int count = 0;
  bool overflow = false, bad_image = false;
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j < n; ++j) {
      const int wj0 = wrap[j], wj1 = wrap[n + j], wj2 = wrap[2 * n + j];
      for (int m0 = -k0; m0 <= k0; ++m0)
        for (int m1 = -k1; m1 <= k1; ++m1)
          for (int m2 = -k2; m2 <= k2; ++m2) {
            const int n0 = m0 + wi0 - wj0, n1 = m1 + wi1 - wj1, n2 = m2 + wi2 - wj2;
            if (j == i && n0 == 0 && n1 == 0 && n2 == 0) continue;
            const double r2 = pair_r2(pos, n, j, xi, yi, zi, n0, n1, n2, box);
            const bool in_a = r2 < rc2_a;
            const bool keep = pass == 0 ? in_a : (!in_a && r2 < rc2_r);
            if (!keep) continue;
            if (n0 < -3 || n0 > 3 || n1 < -3 || n1 > 3 || n2 < -3 || n2 > 3) {
              bad_image = true;
              continue;
            }
            if (count < cap)
              nl[(size_t)count * n + i] = pack_entry(j, n0, n1, n2);
            else
              overflow = true;
            ++count;
          }
    }
    if (pass == 0) cnt_a[i] = min(count, cap);
  }
  cnt_r[i] = min(count, cap);
  if (overflow) flags[kFlagOverflow] = 1;
  if (bad_image) flags[kFlagImage] = 1;
}

// Slot of the reverse entry (i, -n) in atom j's list, for every entry (j, n)
// of atom i.  One thread per (slot, atom).
__global__ void k_reverse(int n, int cap, const uint32_t* __restrict__ nl,
                          const int* __restrict__ cnt_r, int* __restrict__ rev,
                          int* __restrict__ flags) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * cap) return;
  const int i = (int)(idx % (size_t)n);
  const int s = (int)(idx / (size_t)n);
  if (s >= cnt_r[i]) return;
  const uint32_t e = nl[idx];
  const int j = (int)(e & kAtomMask);
  int n0, n1, n2;
  unpack_image(e, n0, n1, n2);
  const uint32_t target = pack_entry(i, -n0, -n1, -n2);
  const int cj = cnt_r[j];
  int found = -1;
  for (int t = 0; t < cj; ++t) {
    if (nl[(size_t)t * n + j] == target) {
      found = t;
      break;
    }
  }
  if (found < 0) {
    flags[kFlagReverse] = 1;
    found = 0;
  }
  rev[idx] = found;
}

__global__ void k_unpack(int n, int cap, const uint32_t* __restrict__ nl, int* __restrict__ nbr,
                         int* __restrict__ img) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * cap) return;
  const uint32_t e = nl[idx];
  int n0, n1, n2;
  unpack_image(e, n0, n1, n2);
  if (nbr) nbr[idx] = (int)(e & kAtomMask);
  if (img) {
    img[3 * idx] = n0;
    img[3 * idx + 1] = n1;
    img[3 * idx + 2] = n2;
  }
}

inline unsigned blocks_for(size_t work, int block) { return (unsigned)((work + block - 1) / block); }

}  // namespace

hipError_t unpack_neighbors(nep_ctx ctx, int* nbr, int* img) {
  const System& s = ctx->sys;
  const size_t ncap = (size_t)s.n * s.cap;
  if (ncap == 0) return hipSuccess;
  k_unpack<<<blocks_for(ncap, kBlock), kBlock, 0, ctx->stream>>>(s.n, s.cap, s.nl.ptr, nbr, img);
  return hipGetLastError();
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

nep_status build_neighbors(nep_ctx ctx, const double* pos_c, bool wrap_in_place) {
  System& s = ctx->sys;
  const int n = s.n;
  hipStream_t st = ctx->stream;
  double* pos = const_cast<double*>(pos_c);  // written only when wrap_in_place
  hipError_t e = hipSuccess;
  const size_t ncap = (size_t)n * s.cap;
  if ((e = s.nl.ensure(ncap)) != hipSuccess || (e = s.rev.ensure(ncap)) != hipSuccess ||
      (e = s.cnt_r.ensure(n)) != hipSuccess || (e = s.cnt_a.ensure(n)) != hipSuccess ||
      (e = s.wrap.ensure((size_t)3 * n)) != hipSuccess)
    return check_hip(ctx, e, "allocating neighbour lists");
  const double rc2_r = s.rc_list_r * s.rc_list_r;
  const double rc2_a = s.rc_list_a * s.rc_list_a;
  if (s.use_cells) {
    const int ncell = s.nc[0] * s.nc[1] * s.nc[2];
    if ((e = s.cell_of.ensure(n)) != hipSuccess || (e = s.cell_cnt.ensure(ncell)) != hipSuccess ||
        (e = s.cell_start.ensure((size_t)ncell + 1)) != hipSuccess ||
        (e = s.cell_fill.ensure(ncell)) != hipSuccess ||
        (e = s.cell_atoms.ensure(n)) != hipSuccess)
      return check_hip(ctx, e, "allocating cell lists");
    k_zero<<<blocks_for(ncell, kBlock), kBlock, 0, st>>>(s.cell_cnt.ptr, ncell);
    k_zero<<<blocks_for(ncell, kBlock), kBlock, 0, st>>>(s.cell_fill.ptr, ncell);
    k_bin<<<blocks_for(n, kBlock), kBlock, 0, st>>>(n, pos, s.box, s.nc[0], s.nc[1], s.nc[2], 1,
                                                    wrap_in_place ? 1 : 0, s.wrap.ptr,
                                                    s.cell_of.ptr, s.cell_cnt.ptr);
    k_scan<<<1, 1024, 0, st>>>(ncell, s.cell_cnt.ptr, s.cell_start.ptr);
    k_fill<<<blocks_for(n, kBlock), kBlock, 0, st>>>(n, s.cell_of.ptr, s.cell_start.ptr,
                                                     s.cell_fill.ptr, s.cell_atoms.ptr);
    k_sort_cells<<<blocks_for(ncell, kBlock), kBlock, 0, st>>>(ncell, s.cell_start.ptr,
                                                               s.cell_atoms.ptr);
    k_build_cells<<<blocks_for(n, kBlock), kBlock, 0, st>>>(
        n, s.cap, pos, s.box, s.nc[0], s.nc[1], s.nc[2], s.wrap.ptr, s.cell_of.ptr,
        s.cell_start.ptr, s.cell_atoms.ptr, rc2_r, rc2_a, s.nl.ptr, s.cnt_r.ptr, s.cnt_a.ptr,
        ctx->flags.ptr);
  } else {
    k_bin<<<blocks_for(n, kBlock), kBlock, 0, st>>>(n, pos, s.box, 1, 1, 1, 0,
                                                    wrap_in_place ? 1 : 0, s.wrap.ptr, nullptr,
                                                    nullptr);
    k_build_all_pairs<<<blocks_for(n, 64), 64, 0, st>>>(
        n, s.cap, pos, s.box, s.kimg[0], s.kimg[1], s.kimg[2], s.wrap.ptr, rc2_r, rc2_a, s.nl.ptr,
        s.cnt_r.ptr, s.cnt_a.ptr, ctx->flags.ptr);
  }
  k_reverse<<<blocks_for(ncap, kBlock), kBlock, 0, st>>>(n, s.cap, s.nl.ptr, s.cnt_r.ptr,
                                                         s.rev.ptr, ctx->flags.ptr);
  return check_hip(ctx, hipGetLastError(), "launching neighbour kernels");
}

}  // namespace nep
