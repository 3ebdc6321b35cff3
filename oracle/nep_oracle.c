/*
 * FP64 CPU oracle for the NEP hot path (Fan et al., "Neuroevolution machine
 * learning potentials", arXiv 2107.08119).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity judge for the GPU path.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code, header or table with the GPU library.
 *
 * Every function follows the paper's definitions literally:
 *   - neighbours: all (j, lattice image n) with |r_j + n.H - r_i| < r_c
 *     (Sec. II A, convention r_ij = r_j - r_i);
 *   - radial functions g_n = (T_n(x)+1)/2 f_c(r), x = 2(r/r_c-1)^2 - 1
 *     (Sec. II C, Eq. g_n; Chebyshev recurrences of Appendix A);
 *   - radial descriptor q_n = sum_j g_n(r_ij)        (Eq. qin);
 *   - angular descriptor q_nl = sum_j sum_k g_n g_n P_l(cos theta_ijk), the
 *     plain O(M^2) double sum, including k = j       (Eq. qinl);
 *   - network x = tanh(W1 q - b1), U_i = w2.x - b2  (Eqs. nn1, nn2);
 *   - partial forces dU_i/dr_ij from the radial and angular derivative
 *     expressions of Sec. II D;
 *   - F_i = sum_j (dU_i/dr_ij - dU_j/dr_ji)          (Sec. II A);
 *   - W_i = sum_j r_ij (x) dU_j/dr_ji, J_i = W_i . v_i (Eq. Wi, Sec. II B);
 *   - loss terms L_e, L_f, L_v, L_1, L_2             (Sec. II E, Eqs. loss*);
 *   - separable NES sampling and update              (Sec. II E 2).
 *
 * Readings of points the paper leaves open (documented with the design):
 *   descriptor order nu = radial n = 0..nR, then angular n-major with l inner;
 *   parameter layout z = [w1 (Nneu x Ndes, row mu), b1, w2, b2];
 *   energy and virial in the loss are per atom (divided by N_s);
 *   virial components xx yy zz xy yz zx;
 *   rank utilities of the natural evolution strategy literature;
 *   Gaussian noise from Philox-4x32-10 counters with the Box-Muller transform.
 *
 * Compile with -ffp-contract=off: the neighbour predicate must be evaluated
 * exactly as written so that neighbour lists can be compared bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

/* 1 eV/Angstrom on 1 amu in Angstrom/fs^2, from e and the atomic mass unit. */
#define OR_ACCEL (1.602176634e-19 / 1.66053906660e-27 * 1.0e-10)

typedef struct {
  double rc_radial, rc_angular;
  int n_max_radial, n_max_angular, l_max, n_neuron;
} or_hyper;

/* ---------------------------------------------------------------- sizes */

/* Eq. N_des: (nR+1) + (nA+1) l_max */
int or_n_des(const or_hyper* h) {
  return (h->n_max_radial + 1) + (h->n_max_angular + 1) * h->l_max;
}

/* Eq. N_par: (N_des + 2) N_neu + 1 */
int or_n_par(const or_hyper* h) { return (or_n_des(h) + 2) * h->n_neuron + 1; }

/* ------------------------------------------------- special functions */

/* Chebyshev polynomials of both kinds by the recurrences of Appendix A:
 * T_0 = 1, T_1 = x, T_n = 2x T_{n-1} - T_{n-2}; U_0 = 1, U_1 = 2x, same rule. */
void or_chebyshev(double x, int nmax, double* T, double* U) {
  for (int n = 0; n <= nmax; ++n) {
    if (n == 0) {
      T[n] = 1.0;
      U[n] = 1.0;
    } else if (n == 1) {
      T[n] = x;
      U[n] = 2.0 * x;
    } else {
      T[n] = 2.0 * x * T[n - 1] - T[n - 2];
      U[n] = 2.0 * x * U[n - 1] - U[n - 2];
    }
  }
}

/* Cutoff function f_c(r) = (1 + cos(pi r / r_c)) / 2 for r <= r_c, else 0,
 * and its derivative. */
static void cutoff(double r, double rc, double* fc, double* dfc) {
  if (r > rc) {
    *fc = 0.0;
    *dfc = 0.0;
    return;
  }
  *fc = 0.5 * (1.0 + cos(OR_PI * r / rc));
  *dfc = -0.5 * OR_PI / rc * sin(OR_PI * r / rc);
}

/* Radial functions g_n(r) = (T_n(x) + 1)/2 f_c(r) with x = 2(r/r_c - 1)^2 - 1
 * (Eq. g_n), n = 0..nmax, and dg_n/dr using dT_n/dx = n U_{n-1}(x). */
void or_radial_basis(double r, double rc, int nmax, double* g, double* dg) {
  double T[64], U[64];
  double fc, dfc;
  cutoff(r, rc, &fc, &dfc);
  double t = r / rc - 1.0;
  double x = 2.0 * t * t - 1.0;
  double dxdr = 4.0 * t / rc;
  or_chebyshev(x, nmax, T, U);
  for (int n = 0; n <= nmax; ++n) {
    double dT = (n == 0) ? 0.0 : n * U[n - 1];
    g[n] = 0.5 * (T[n] + 1.0) * fc;
    dg[n] = 0.5 * dT * dxdr * fc + 0.5 * (T[n] + 1.0) * dfc;
  }
}

/* Legendre polynomials by Bonnet's recurrence (l+1) P_{l+1} = (2l+1) c P_l - l P_{l-1},
 * and derivatives by P'_{l+1} = P'_{l-1} + (2l+1) P_l. */
void or_legendre(double c, int lmax, double* P, double* dP) {
  P[0] = 1.0;
  dP[0] = 0.0;
  if (lmax >= 1) {
    P[1] = c;
    dP[1] = 1.0;
  }
  for (int l = 1; l < lmax; ++l) {
    P[l + 1] = ((2 * l + 1) * c * P[l] - l * P[l - 1]) / (l + 1);
    dP[l + 1] = dP[l - 1] + (2 * l + 1) * P[l];
  }
}

/* ------------------------------------------------------- neighbours */

static void invert3(const double* H, double* Hi) {
  double a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7],
         k = H[8];
  double det = a * (e * k - f * h) - b * (d * k - f * g) + c * (d * h - e * g);
  Hi[0] = (e * k - f * h) / det;
  Hi[1] = (c * h - b * k) / det;
  Hi[2] = (b * f - c * e) / det;
  Hi[3] = (f * g - d * k) / det;
  Hi[4] = (a * k - c * g) / det;
  Hi[5] = (c * d - a * f) / det;
  Hi[6] = (d * h - e * g) / det;
  Hi[7] = (b * g - a * h) / det;
  Hi[8] = (a * e - b * d) / det;
}

/* Distance between opposite faces of the cell for each cell vector. */
static void face_widths(const double* H, double* w) {
  const double* A = H;
  const double* B = H + 3;
  const double* C = H + 6;
  double bc[3] = {B[1] * C[2] - B[2] * C[1], B[2] * C[0] - B[0] * C[2], B[0] * C[1] - B[1] * C[0]};
  double ca[3] = {C[1] * A[2] - C[2] * A[1], C[2] * A[0] - C[0] * A[2], C[0] * A[1] - C[1] * A[0]};
  double ab[3] = {A[1] * B[2] - A[2] * B[1], A[2] * B[0] - A[0] * B[2], A[0] * B[1] - A[1] * B[0]};
  double vol = fabs(A[0] * bc[0] + A[1] * bc[1] + A[2] * bc[2]);
  w[0] = vol / sqrt(bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
  w[1] = vol / sqrt(ca[0] * ca[0] + ca[1] * ca[1] + ca[2] * ca[2]);
  w[2] = vol / sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
}

/* The pair displacement r_ij = r_j + n.H - r_i, evaluated in exactly this
 * order (shift summed over cell vectors a, b, c; then added to r_j - r_i). */
static void pair_displacement(const double* pos, const double* H, int i, int j, int n0, int n1,
                              int n2, double* d) {
  for (int c = 0; c < 3; ++c) {
    double shift = ((double)n0 * H[c] + (double)n1 * H[3 + c]) + (double)n2 * H[6 + c];
    d[c] = (pos[3 * j + c] - pos[3 * i + c]) + shift;
  }
}

static double norm2(const double* d) { return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]; }

typedef struct {
  int cap;
  int* cnt; /* [N] */
  int* j;   /* [N][cap] */
  int* img; /* [N][cap][3] */
} or_list;

static void list_free(or_list* L) {
  free(L->cnt);
  free(L->j);
  free(L->img);
  L->cnt = L->j = L->img = NULL;
}

/* For every atom i with need[i] != 0, list all (j, n) with 0 < |r_ij| < rc.
 * Candidates come from a cell grid in fractional coordinates (a plain filter;
 * the predicate alone decides membership).  Returns 0, or -1 if some atom has
 * more than cap neighbours, or -3 on allocation failure. */
static int build_list(int N, const double* pos, const double* H, double rc,
                      const unsigned char* need, int cap, or_list* L) {
  double Hi[9], wid[3];
  invert3(H, Hi);
  face_widths(H, wid);
  int nc[3];
  double t[3];
  for (int a = 0; a < 3; ++a) {
    t[a] = rc / wid[a] * (1.0 + 1e-12) + 1e-12;
    nc[a] = (int)floor(wid[a] / (rc * (1.0 + 1e-9)));
    if (nc[a] < 3) nc[a] = 1; /* thin direction: no filtering along it */
  }
  double* frac = (double*)malloc(sizeof(double) * 3 * (size_t)(N > 0 ? N : 1));
  int* cell = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
  int ncell = nc[0] * nc[1] * nc[2];
  int* start = (int*)calloc((size_t)ncell + 1, sizeof(int));
  int* members = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
  L->cap = cap;
  L->cnt = (int*)calloc((size_t)(N > 0 ? N : 1), sizeof(int));
  L->j = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1) * cap);
  L->img = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1) * cap * 3);
  if (!frac || !cell || !start || !members || !L->cnt || !L->j || !L->img) {
    free(frac);
    free(cell);
    free(start);
    free(members);
    list_free(L);
    return -3;
  }
  for (int i = 0; i < N; ++i) {
    int ci[3];
    for (int a = 0; a < 3; ++a) {
      double s = pos[3 * i] * Hi[a] + pos[3 * i + 1] * Hi[3 + a] + pos[3 * i + 2] * Hi[6 + a];
      frac[3 * i + a] = s;
      double sw = s - floor(s);
      int c = (int)(sw * nc[a]);
      if (c >= nc[a]) c = nc[a] - 1;
      if (c < 0) c = 0;
      ci[a] = c;
    }
    cell[i] = (ci[2] * nc[1] + ci[1]) * nc[0] + ci[0];
    start[cell[i] + 1]++;
  }
  for (int c = 0; c < ncell; ++c) start[c + 1] += start[c];
  {
    int* fill = (int*)calloc((size_t)ncell, sizeof(int));
    for (int i = 0; i < N; ++i) members[start[cell[i]] + fill[cell[i]]++] = i;
    free(fill);
  }
  int overflow = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : overflow)
  for (int i = 0; i < N; ++i) {
    if (!need[i]) continue;
    int c0 = cell[i] % nc[0];
    int c1 = (cell[i] / nc[0]) % nc[1];
    int c2 = cell[i] / (nc[0] * nc[1]);
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = (nc[a] >= 3) ? -1 : 0;
      hi[a] = (nc[a] >= 3) ? 1 : 0;
    }
    int count = 0;
    for (int o2 = lo[2]; o2 <= hi[2]; ++o2)
      for (int o1 = lo[1]; o1 <= hi[1]; ++o1)
        for (int o0 = lo[0]; o0 <= hi[0]; ++o0) {
          int d0 = ((c0 + o0) % nc[0] + nc[0]) % nc[0];
          int d1 = ((c1 + o1) % nc[1] + nc[1]) % nc[1];
          int d2 = ((c2 + o2) % nc[2] + nc[2]) % nc[2];
          int cc = (d2 * nc[1] + d1) * nc[0] + d0;
          for (int m = start[cc]; m < start[cc + 1]; ++m) {
            int j = members[m];
            int nlo[3], nhi[3];
            for (int a = 0; a < 3; ++a) {
              double ds = frac[3 * j + a] - frac[3 * i + a];
              nlo[a] = (int)ceil(-ds - t[a]);
              nhi[a] = (int)floor(-ds + t[a]);
            }
            for (int n0 = nlo[0]; n0 <= nhi[0]; ++n0)
              for (int n1 = nlo[1]; n1 <= nhi[1]; ++n1)
                for (int n2 = nlo[2]; n2 <= nhi[2]; ++n2) {
                  if (j == i && n0 == 0 && n1 == 0 && n2 == 0) continue;
                  double d[3];
                  pair_displacement(pos, H, i, j, n0, n1, n2, d);
                  if (norm2(d) < rc * rc) {
                    if (count < cap) {
                      L->j[(size_t)i * cap + count] = j;
                      L->img[((size_t)i * cap + count) * 3 + 0] = n0;
                      L->img[((size_t)i * cap + count) * 3 + 1] = n1;
                      L->img[((size_t)i * cap + count) * 3 + 2] = n2;
                    } else {
                      overflow = 1;
                    }
                    count++;
                  }
                }
          }
        }
    L->cnt[i] = count < cap ? count : cap;
  }
  free(frac);
  free(cell);
  free(start);
  free(members);
  return overflow ? -1 : 0;
}

/* Neighbour list of every atom: for each i, its count and (j, n0, n1, n2)
 * entries in an unspecified order.  pos is [N][3], H holds the cell vectors
 * as rows.  Returns 0, -1 on capacity overflow, -3 on allocation failure. */
int or_neighbors(int N, const double* pos, const double* H, double rc, int cap, int* cnt,
                 int* j_out, int* img_out) {
  unsigned char* need = (unsigned char*)malloc((size_t)(N > 0 ? N : 1));
  if (!need) return -3;
  memset(need, 1, (size_t)(N > 0 ? N : 1));
  or_list L;
  int rcode = build_list(N, pos, H, rc, need, cap, &L);
  free(need);
  if (rcode == -3) return rcode;
  memcpy(cnt, L.cnt, sizeof(int) * (size_t)N);
  memcpy(j_out, L.j, sizeof(int) * (size_t)N * cap);
  memcpy(img_out, L.img, sizeof(int) * (size_t)N * cap * 3);
  list_free(&L);
  return rcode;
}

/* -------------------------------------------------- NEP, per atom */

/* Geometry of atom i's listed pairs: displacements d [cnt][3], distances r,
 * species weights w, and the angular radial functions g_n, g_n' with r_c^A
 * (zero beyond it), species weight included.
 *
 * Multicomponent systems (Sec. II C, multicomponent paragraph): the cutoff
 * function of pair (i, j) is multiplied by sqrt(Z_i Z_j), Z = atomic number,
 * so every radial function g_n(r_ij) and its derivative carries that factor.
 * Without species (Z == NULL) the factor is 1. */
typedef struct {
  int cnt;
  double* d;
  double* r;
  double* w;
  double* gA;
  double* dgA;
} or_geom;

static void geom_free(or_geom* G) {
  free(G->d);
  free(G->r);
  free(G->w);
  free(G->gA);
  free(G->dgA);
}

static int geom_build(const or_hyper* hp, const double* pos, const double* H, const int* Z,
                      int i, int cnt, const int* jl, const int* img, or_geom* G) {
  const int nA = hp->n_max_angular;
  const size_t m = (size_t)(cnt > 0 ? cnt : 1);
  G->cnt = cnt;
  G->d = (double*)malloc(sizeof(double) * 3 * m);
  G->r = (double*)malloc(sizeof(double) * m);
  G->w = (double*)malloc(sizeof(double) * m);
  G->gA = (double*)malloc(sizeof(double) * (nA + 1) * m);
  G->dgA = (double*)malloc(sizeof(double) * (nA + 1) * m);
  if (!G->d || !G->r || !G->w || !G->gA || !G->dgA) {
    geom_free(G);
    return -3;
  }
  for (int s = 0; s < cnt; ++s) {
    pair_displacement(pos, H, i, jl[s], img[3 * s], img[3 * s + 1], img[3 * s + 2], G->d + 3 * s);
    G->r[s] = sqrt(norm2(G->d + 3 * s));
    G->w[s] = Z ? sqrt((double)Z[i] * (double)Z[jl[s]]) : 1.0;
    if (G->r[s] < hp->rc_angular) {
      or_radial_basis(G->r[s], hp->rc_angular, nA, G->gA + (nA + 1) * s, G->dgA + (nA + 1) * s);
      for (int n = 0; n <= nA; ++n) {
        G->gA[(nA + 1) * s + n] *= G->w[s];
        G->dgA[(nA + 1) * s + n] *= G->w[s];
      }
    } else {
      for (int n = 0; n <= nA; ++n) G->gA[(nA + 1) * s + n] = G->dgA[(nA + 1) * s + n] = 0.0;
    }
  }
  return 0;
}

/* Descriptor q (Eqs. qin, qinl; the angular double sum includes k = j). */
static void descriptor(const or_hyper* hp, const or_geom* G, double* q) {
  const int nR = hp->n_max_radial, nA = hp->n_max_angular, lmax = hp->l_max;
  const int ndes = or_n_des(hp);
  const double rcR = hp->rc_radial, rcA = hp->rc_angular;
  const double* d = G->d;
  const double* r = G->r;
  double g[64], dg[64], P[16], dP[16];
  for (int v = 0; v < ndes; ++v) q[v] = 0.0;
  for (int s = 0; s < G->cnt; ++s) {
    if (r[s] >= rcR) continue;
    or_radial_basis(r[s], rcR, nR, g, dg);
    for (int n = 0; n <= nR; ++n) q[n] += G->w[s] * g[n];
  }
  for (int s = 0; s < G->cnt; ++s) {
    if (r[s] >= rcA) continue;
    for (int t = 0; t < G->cnt; ++t) {
      if (r[t] >= rcA) continue;
      double c = (d[3 * s] * d[3 * t] + d[3 * s + 1] * d[3 * t + 1] + d[3 * s + 2] * d[3 * t + 2]) /
                 (r[s] * r[t]);
      or_legendre(c, lmax, P, dP);
      for (int n = 0; n <= nA; ++n)
        for (int l = 1; l <= lmax; ++l)
          q[(nR + 1) + n * lmax + (l - 1)] +=
              G->gA[(nA + 1) * s + n] * G->gA[(nA + 1) * t + n] * P[l];
    }
  }
}

/* Network (Eqs. nn1, nn2): U = sum_mu w2 tanh(a_mu) - b2 with
 * a_mu = sum_nu w1[mu][nu] q_nu - b1[mu]; dU/dq_nu = sum_mu w2 (1 - x^2) w1[mu][nu].
 * x (the hidden state, [N_neu]) may be NULL. */
static void network(const or_hyper* hp, const double* z, const double* q, double* U, double* dUdq,
                    double* x_out) {
  const int ndes = or_n_des(hp), nneu = hp->n_neuron;
  const double* w1 = z;
  const double* b1 = z + nneu * ndes;
  const double* w2 = b1 + nneu;
  const double b2 = w2[nneu];
  double u = 0.0;
  for (int v = 0; v < ndes; ++v) dUdq[v] = 0.0;
  for (int m = 0; m < nneu; ++m) {
    double a = -b1[m];
    for (int v = 0; v < ndes; ++v) a += w1[m * ndes + v] * q[v];
    double x = tanh(a);
    if (x_out) x_out[m] = x;
    u += w2[m] * x;
    for (int v = 0; v < ndes; ++v) dUdq[v] += w2[m] * (1.0 - x * x) * w1[m * ndes + v];
  }
  *U = u - b2;
}

/* Partial forces p_s = sum_nu dUdq_nu dq_nu/dr_ij for every listed pair s,
 * from the radial and angular derivative expressions of Sec. II D. */
static void partials(const or_hyper* hp, const or_geom* G, const double* dUdq, double* p) {
  const int nR = hp->n_max_radial, nA = hp->n_max_angular, lmax = hp->l_max;
  const double rcR = hp->rc_radial, rcA = hp->rc_angular;
  const double* d = G->d;
  const double* r = G->r;
  const int cnt = G->cnt;
  double g[64], dg[64], P[16], dP[16];
  for (int s = 0; s < cnt; ++s) {
    double* ps = p + 3 * s;
    ps[0] = ps[1] = ps[2] = 0.0;
    double rs = r[s];
    double us[3] = {d[3 * s] / rs, d[3 * s + 1] / rs, d[3 * s + 2] / rs};
    if (rs < rcR) {
      or_radial_basis(rs, rcR, nR, g, dg);
      double f = 0.0;
      for (int n = 0; n <= nR; ++n) f += dUdq[n] * G->w[s] * dg[n];
      for (int c = 0; c < 3; ++c) ps[c] += f * us[c];
    }
    if (rs < rcA) {
      for (int t = 0; t < cnt; ++t) {
        if (r[t] >= rcA) continue;
        double ut[3] = {d[3 * t] / r[t], d[3 * t + 1] / r[t], d[3 * t + 2] / r[t]};
        /* same cosine expression as the descriptor sum */
        double c = (d[3 * s] * d[3 * t] + d[3 * s + 1] * d[3 * t + 1] + d[3 * s + 2] * d[3 * t + 2]) /
                   (r[s] * r[t]);
        or_legendre(c, lmax, P, dP);
        for (int n = 0; n <= nA; ++n) {
          double gs = G->gA[(nA + 1) * s + n], dgs = G->dgA[(nA + 1) * s + n];
          double gt = G->gA[(nA + 1) * t + n];
          for (int l = 1; l <= lmax; ++l) {
            double w = dUdq[(nR + 1) + n * lmax + (l - 1)];
            double a1 = 2.0 * dgs * gt * P[l];
            double a2 = 2.0 * gs * gt * dP[l] / rs;
            for (int cc = 0; cc < 3; ++cc) ps[cc] += w * (a1 * us[cc] + a2 * (ut[cc] - us[cc] * c));
          }
        }
      }
    }
  }
}

/* Descriptor, network and partial forces of atom i (p is [cnt][3]). */
static void atom_terms(const or_hyper* hp, const double* z, const double* pos, const double* H,
                       const int* Z, int i, int cnt, const int* jl, const int* img, double* q,
                       double* U, double* dUdq, double* p) {
  or_geom G;
  if (geom_build(hp, pos, H, Z, i, cnt, jl, img, &G)) return;
  descriptor(hp, &G, q);
  network(hp, z, q, U, dUdq, NULL);
  partials(hp, &G, dUdq, p);
  geom_free(&G);
}

/* Index of the reverse pair (j -> i, image -n) in atom j's list, or -1. */
static int find_reverse(const or_list* L, int i, int j, const int* n) {
  for (int t = 0; t < L->cnt[j]; ++t) {
    const int* m = L->img + ((size_t)j * L->cap + t) * 3;
    if (L->j[(size_t)j * L->cap + t] == i && m[0] == -n[0] && m[1] == -n[1] && m[2] == -n[2])
      return t;
  }
  return -1;
}

/* Energies, forces, full per-atom virials and heat currents of the atoms in
 * sel (all atoms when sel is NULL; then n_sel must equal N).
 *   pos [N][3], H [3][3] rows = cell vectors, vel [N][3] or NULL, z [N_par];
 *   outputs indexed by position in sel: U [n_sel], F [n_sel][3],
 *   W [n_sel][9] row-major (W_ab = sum_j (r_ij)_a (dU_j/dr_ji)_b),
 *   J [n_sel][3] (zero when vel is NULL), q [n_sel][N_des] (may be NULL);
 *   Z [N] atomic numbers of a multicomponent system, or NULL (one species).
 * Returns 0, -1 on neighbour capacity overflow, -2 on a missing reverse pair,
 * -3 on allocation failure. */
int or_nep_eval_species(const or_hyper* hp, const double* z, int N, const double* pos,
                        const double* H, const int* Z, const double* vel, int n_sel,
                        const int* sel, int cap, double* U, double* F, double* W, double* J,
                        double* q_out) {
  const int ndes = or_n_des(hp);
  double rc = hp->rc_radial > hp->rc_angular ? hp->rc_radial : hp->rc_angular;
  unsigned char* need = (unsigned char*)calloc((size_t)(N > 0 ? N : 1), 1);
  if (!need) return -3;
  for (int k = 0; k < n_sel; ++k) need[sel ? sel[k] : k] = 1;
  or_list L1;
  int rcode = build_list(N, pos, H, rc, need, cap, &L1);
  if (rcode) {
    free(need);
    if (rcode != -3) list_free(&L1);
    return rcode;
  }
  /* the reverse partials need the neighbours' own terms */
  for (int k = 0; k < n_sel; ++k) {
    int i = sel ? sel[k] : k;
    for (int s = 0; s < L1.cnt[i]; ++s) need[L1.j[(size_t)i * cap + s]] = 1;
  }
  list_free(&L1);
  or_list L;
  rcode = build_list(N, pos, H, rc, need, cap, &L);
  if (rcode) {
    free(need);
    if (rcode != -3) list_free(&L);
    return rcode;
  }
  double* p = (double*)malloc(sizeof(double) * 3 * (size_t)N * cap);
  double* Uall = (double*)malloc(sizeof(double) * (size_t)N);
  double* qall = (double*)malloc(sizeof(double) * (size_t)N * ndes);
  if (!p || !Uall || !qall) {
    free(p);
    free(Uall);
    free(qall);
    free(need);
    list_free(&L);
    return -3;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < N; ++i) {
    if (!need[i]) continue;
    double dUdq[256];
    atom_terms(hp, z, pos, H, Z, i, L.cnt[i], L.j + (size_t)i * cap, L.img + (size_t)i * cap * 3,
               qall + (size_t)i * ndes, Uall + i, dUdq, p + (size_t)i * cap * 3);
  }
  int missing = 0;
#pragma omp parallel for schedule(static) reduction(| : missing)
  for (int k = 0; k < n_sel; ++k) {
    int i = sel ? sel[k] : k;
    double f[3] = {0, 0, 0}, w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = 0; s < L.cnt[i]; ++s) {
      int j = L.j[(size_t)i * cap + s];
      const int* n = L.img + ((size_t)i * cap + s) * 3;
      int t = find_reverse(&L, i, j, n);
      if (t < 0) {
        missing = 1;
        continue;
      }
      const double* pij = p + ((size_t)i * cap + s) * 3;
      const double* pji = p + ((size_t)j * cap + t) * 3;
      double d[3];
      pair_displacement(pos, H, i, j, n[0], n[1], n[2], d);
      for (int a = 0; a < 3; ++a) {
        f[a] += pij[a] - pji[a];
        for (int b = 0; b < 3; ++b) w[3 * a + b] += d[a] * pji[b];
      }
    }
    U[k] = Uall[i];
    for (int a = 0; a < 3; ++a) F[3 * k + a] = f[a];
    if (W)
      for (int a = 0; a < 9; ++a) W[9 * k + a] = w[a];
    if (J)
      for (int a = 0; a < 3; ++a)
        J[3 * k + a] =
            vel ? w[3 * a] * vel[3 * i] + w[3 * a + 1] * vel[3 * i + 1] + w[3 * a + 2] * vel[3 * i + 2]
                : 0.0;
    if (q_out)
      for (int v = 0; v < ndes; ++v) q_out[(size_t)k * ndes + v] = qall[(size_t)i * ndes + v];
  }
  free(p);
  free(Uall);
  free(qall);
  free(need);
  list_free(&L);
  return missing ? -2 : 0;
}

/* or_nep_eval_species of a one-species system. */
int or_nep_eval(const or_hyper* hp, const double* z, int N, const double* pos, const double* H,
                const double* vel, int n_sel, const int* sel, int cap, double* U, double* F,
                double* W, double* J, double* q_out) {
  return or_nep_eval_species(hp, z, N, pos, H, NULL, vel, n_sel, sel, cap, U, F, W, J, q_out);
}

/* ------------------------------------------------- parameter gradient */

/* Gradient with respect to z of
 *   G(z) = sum_s gE[s] E_s(z) + sum_i gF_i . F_i(z)
 * over a set of structures laid out as in or_loss (gF is [sum N][3]).
 * Energy part: dU_a/dz from Eqs. nn1, nn2.  Force part: by Sec. II A,
 * sum_i gF_i . F_i = sum over listed pairs (a, j) of p_aj . (gF_a - gF_j), and
 * p_aj = sum_nu dU_a/dq_nu dq_nu/dr_aj, where dq_nu/dr_aj is evaluated with
 * the partial-force expressions of Sec. II D for a unit vector dU/dq = e_nu;
 * only dU_a/dq_nu depends on z, through the network.
 * Returns 0 or a negative error code. */
int or_grad_params(const or_hyper* hp, const double* z, int n_struct, const int* n_atoms,
                   const double* boxes, const double* pos, const double* gE, const double* gF,
                   int cap, double* grad) {
  const int ndes = or_n_des(hp), nneu = hp->n_neuron, npar = or_n_par(hp);
  const double* w1 = z;
  const double* w2 = z + nneu * ndes + nneu;
  const double rc = hp->rc_radial > hp->rc_angular ? hp->rc_radial : hp->rc_angular;
  for (int k = 0; k < npar; ++k) grad[k] = 0.0;
  size_t off = 0;
  int status = 0;
  for (int st = 0; st < n_struct && status == 0; ++st) {
    const int n = n_atoms[st];
    const double* P = pos + 3 * off;
    const double* H = boxes + 9 * st;
    const double* gFs = gF + 3 * off;
    unsigned char* need = (unsigned char*)malloc((size_t)n);
    if (!need) return -3;
    memset(need, 1, (size_t)n);
    or_list L;
    int rcode = build_list(n, P, H, rc, need, cap, &L);
    free(need);
    if (rcode) {
      if (rcode != -3) list_free(&L);
      return rcode;
    }
#pragma omp parallel
    {
      double q[256], dUdq[256], x[4096], v[256], e[256];
      double* mine = (double*)calloc((size_t)npar, sizeof(double));
      double* gw1 = mine;
      double* gb1 = mine + nneu * ndes;
      double* gw2 = gb1 + nneu;
      double* gb2 = gw2 + nneu;
#pragma omp for schedule(static)
      for (int a = 0; a < n; ++a) {
        or_geom G;
        const int cnt = L.cnt[a];
        const int* jl = L.j + (size_t)a * cap;
        double* D = (double*)malloc(sizeof(double) * 3 * (size_t)(cnt > 0 ? cnt : 1));
        if (!mine || !D || geom_build(hp, P, H, NULL, a, cnt, jl, L.img + (size_t)a * cap * 3, &G)) {
          free(D);
#pragma omp atomic write
          status = -3;
          continue;
        }
        double U;
        descriptor(hp, &G, q);
        network(hp, z, q, &U, dUdq, x);
        /* energy part */
        for (int m = 0; m < nneu; ++m) {
          const double sm = 1.0 - x[m] * x[m];
          for (int nu = 0; nu < ndes; ++nu) gw1[m * ndes + nu] += gE[st] * w2[m] * sm * q[nu];
          gb1[m] += gE[st] * (-w2[m] * sm);
          gw2[m] += gE[st] * x[m];
        }
        gb2[0] += -gE[st];
        /* force part: v_nu = sum over pairs of dq_nu/dr_aj . (gF_a - gF_j) */
        for (int nu = 0; nu < ndes; ++nu) {
          for (int k = 0; k < ndes; ++k) e[k] = k == nu ? 1.0 : 0.0;
          partials(hp, &G, e, D);
          double acc = 0.0;
          for (int sl = 0; sl < cnt; ++sl) {
            const int j = jl[sl];
            for (int c = 0; c < 3; ++c) acc += D[3 * sl + c] * (gFs[3 * a + c] - gFs[3 * j + c]);
          }
          v[nu] = acc;
        }
        free(D);
        /* d(dU_a/dq_nu)/dz contracted with v */
        for (int m = 0; m < nneu; ++m) {
          const double sm = 1.0 - x[m] * x[m];
          double wv = 0.0;
          for (int nu = 0; nu < ndes; ++nu) wv += w1[m * ndes + nu] * v[nu];
          gw2[m] += sm * wv;
          gb1[m] += 2.0 * w2[m] * x[m] * sm * wv;
          for (int kap = 0; kap < ndes; ++kap)
            gw1[m * ndes + kap] += w2[m] * (-2.0 * x[m] * sm * q[kap] * wv + sm * v[kap]);
        }
        geom_free(&G);
      }
#pragma omp critical
      {
        if (mine)
          for (int k = 0; k < npar; ++k) grad[k] += mine[k];
      }
      free(mine);
    }
    list_free(&L);
    off += (size_t)n;
  }
  return status;
}

/* --------------------------------------------------- molecular dynamics */

/* F_i += F_e . W_i for every atom (W_i row-major, (W_i)_ab at 3a + b). */
static void add_driving_force(int N, const double* fe, const double* W, double* F) {
  for (int i = 0; i < N; ++i) {
    const double* w = W + 9 * (size_t)i;
    for (int b = 0; b < 3; ++b) F[3 * (size_t)i + b] += fe[0] * w[b] + fe[1] * w[3 + b] + fe[2] * w[6 + b];
  }
}

/* Velocity-Verlet trajectory with exact cutoffs at every step.
 * pos/vel [N][3] are updated in place; thermo [n_steps][5] receives
 * E_pot, E_kin (eV), and the total heat current sum_i J_i (3 components)
 * after each step.  mass in amu (per atom from masses [N] when that is not
 * NULL), dt in fs; Z [N] atomic numbers of a multicomponent system or NULL.
 * With fe != NULL every atom also
 * feels the homogeneous driving force of the HNEMD method (Sec. II B):
 * F_i^ext = F_e . W_i, i.e. (F_i^ext)_b = sum_a (F_e)_a (W_i)_ab, with F_e in
 * 1/Angstrom; fe == NULL is plain NVE. */
int or_md_species(const or_hyper* hp, const double* z, int N, double* pos, const double* H,
                  const int* Z, const double* masses, double* vel, double mass, double dt,
                  int n_steps, int cap, const double* fe, double* thermo) {
  double* U = (double*)malloc(sizeof(double) * (size_t)N);
  double* F = (double*)malloc(sizeof(double) * 3 * (size_t)N);
  double* W = (double*)malloc(sizeof(double) * 9 * (size_t)N);
  if (!U || !F || !W) {
    free(U);
    free(F);
    free(W);
    return -3;
  }
  int rcode = or_nep_eval_species(hp, z, N, pos, H, Z, NULL, N, NULL, cap, U, F, W, NULL, NULL);
  if (rcode == 0 && fe) add_driving_force(N, fe, W, F);
  for (int step = 0; step < n_steps && rcode == 0; ++step) {
    for (int i = 0; i < 3 * N; ++i) {
      vel[i] += 0.5 * dt * (OR_ACCEL / (masses ? masses[i / 3] : mass)) * F[i];
      pos[i] += dt * vel[i];
    }
    rcode = or_nep_eval_species(hp, z, N, pos, H, Z, NULL, N, NULL, cap, U, F, W, NULL, NULL);
    if (rcode) break;
    if (fe) add_driving_force(N, fe, W, F);
    for (int i = 0; i < 3 * N; ++i)
      vel[i] += 0.5 * dt * (OR_ACCEL / (masses ? masses[i / 3] : mass)) * F[i];
    /* heat current J_i = W_i . v_i with the end-of-step velocities */
    double ep = 0.0, ek = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
    for (int i = 0; i < N; ++i) {
      const double* w = W + 9 * (size_t)i;
      const double* v = vel + 3 * (size_t)i;
      ep += U[i];
      ek += 0.5 * (masses ? masses[i] : mass) * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) /
            OR_ACCEL;
      j0 += w[0] * v[0] + w[1] * v[1] + w[2] * v[2];
      j1 += w[3] * v[0] + w[4] * v[1] + w[5] * v[2];
      j2 += w[6] * v[0] + w[7] * v[1] + w[8] * v[2];
    }
    thermo[5 * step + 0] = ep;
    thermo[5 * step + 1] = ek;
    thermo[5 * step + 2] = j0;
    thermo[5 * step + 3] = j1;
    thermo[5 * step + 4] = j2;
  }
  free(U);
  free(F);
  free(W);
  return rcode;
}

/* One species, one mass. */
int or_md_driven(const or_hyper* hp, const double* z, int N, double* pos, const double* H,
                 double* vel, double mass, double dt, int n_steps, int cap, const double* fe,
                 double* thermo) {
  return or_md_species(hp, z, N, pos, H, NULL, NULL, vel, mass, dt, n_steps, cap, fe, thermo);
}

/* Velocity-Verlet NVE: or_md_driven without a driving force. */
int or_md_nve(const or_hyper* hp, const double* z, int N, double* pos, const double* H,
              double* vel, double mass, double dt, int n_steps, int cap, double* thermo) {
  return or_md_driven(hp, z, N, pos, H, vel, mass, dt, n_steps, cap, NULL, thermo);
}

/* ------------------------------------------------------------ loss */

/* Loss of one parameter vector over a training set (Eq. loss and the five
 * terms that follow it).  Structures are concatenated: n_atoms [S],
 * boxes [S][9], pos [sum N][3], E_tar [S] (total energy), F_tar [sum N][3],
 * W_tar [S][6] (total virial xx yy zz xy yz zx), has_virial [S].
 * Energies and virials are compared per atom.  lambda = (e, f, v, 1, 2).
 * out = (L, L_e, L_f, L_v, L_1, L_2). */
int or_loss(const or_hyper* hp, const double* z, int n_struct, const int* n_atoms,
            const double* boxes, const double* pos, const double* E_tar, const double* F_tar,
            const double* W_tar, const unsigned char* has_virial, const double* lambda, int cap,
            double* out) {
  static const int comp[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {1, 2}, {2, 0}};
  const int npar = or_n_par(hp);
  double se = 0.0, sf = 0.0, sv = 0.0;
  long nv = 0, ntot = 0;
  size_t off = 0;
  for (int s = 0; s < n_struct; ++s) {
    int n = n_atoms[s];
    double* U = (double*)malloc(sizeof(double) * (size_t)n);
    double* F = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* W = (double*)malloc(sizeof(double) * 9 * (size_t)n);
    if (!U || !F || !W) {
      free(U);
      free(F);
      free(W);
      return -3;
    }
    int rcode = or_nep_eval(hp, z, n, pos + 3 * off, boxes + 9 * s, NULL, n, NULL, cap, U, F, W,
                            NULL, NULL);
    if (rcode) {
      free(U);
      free(F);
      free(W);
      return rcode;
    }
    double e = 0.0, w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < n; ++i) {
      e += U[i];
      for (int a = 0; a < 9; ++a) w[a] += W[9 * i + a];
      for (int a = 0; a < 3; ++a) {
        double df = F[3 * i + a] - F_tar[3 * (off + i) + a];
        sf += df * df;
      }
    }
    double de = e / n - E_tar[s] / n;
    se += de * de;
    if (has_virial[s]) {
      for (int c = 0; c < 6; ++c) {
        double dv = w[3 * comp[c][0] + comp[c][1]] / n - W_tar[6 * s + c] / n;
        sv += dv * dv;
      }
      nv++;
    }
    ntot += n;
    off += (size_t)n;
    free(U);
    free(F);
    free(W);
  }
  double l1 = 0.0, l2 = 0.0;
  for (int k = 0; k < npar; ++k) {
    l1 += fabs(z[k]);
    l2 += z[k] * z[k];
  }
  out[1] = sqrt(se / n_struct);
  out[2] = sqrt(sf / (3.0 * ntot));
  out[3] = nv ? sqrt(sv / (6.0 * nv)) : 0.0;
  out[4] = l1 / npar;
  out[5] = sqrt(l2 / npar);
  out[0] = lambda[0] * out[1] + lambda[1] * out[2] + lambda[2] * out[3] + lambda[3] * out[4] +
           lambda[4] * out[5];
  return 0;
}

/* ------------------------------------------------------------- SNES */

/* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
 * Philox S-box with multipliers 0xD2511F53 and 0xCD9E8D57 and the key
 * schedule constants 0x9E3779B9 and 0xBB67AE85. */
void or_philox4x32_10(const uint32_t* ctr_in, const uint32_t* key_in, uint32_t* out) {
  uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* Standard normal numbers r_k for individual k of generation gen: counter
 * (b, k, gen, 0) with key (seed low, seed high) gives four uniforms
 * u = (x + 1/2) 2^-32, turned into four normals by the Box-Muller transform
 * (pairs (u0,u1) and (u2,u3)); they fill parameters 4b..4b+3.
 * z_k = m + s . r_k.  r and z are rounded to float32. */
void or_snes_sample(int n_par, int n_pop, const float* m, const float* s, uint64_t seed, int gen,
                    float* r_out, float* z_out) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int k = 0; k < n_pop; ++k) {
    for (int b = 0; 4 * b < n_par; ++b) {
      uint32_t ctr[4] = {(uint32_t)b, (uint32_t)k, (uint32_t)gen, 0u};
      uint32_t x[4];
      or_philox4x32_10(ctr, key, x);
      double u[4];
      for (int t = 0; t < 4; ++t) u[t] = ((double)x[t] + 0.5) * (1.0 / 4294967296.0);
      double nrm[4];
      double rad0 = sqrt(-2.0 * log(u[0])), rad1 = sqrt(-2.0 * log(u[2]));
      nrm[0] = rad0 * cos(2.0 * OR_PI * u[1]);
      nrm[1] = rad0 * sin(2.0 * OR_PI * u[1]);
      nrm[2] = rad1 * cos(2.0 * OR_PI * u[3]);
      nrm[3] = rad1 * sin(2.0 * OR_PI * u[3]);
      for (int t = 0; t < 4 && 4 * b + t < n_par; ++t) {
        int v = 4 * b + t;
        float rv = (float)nrm[t];
        r_out[(size_t)k * n_par + v] = rv;
        z_out[(size_t)k * n_par + v] = (float)((double)m[v] + (double)s[v] * (double)rv);
      }
    }
  }
}

/* Rank-based utilities of the natural evolution strategy literature:
 * u_k = max(0, ln(P/2 + 1) - ln k) / sum_j max(0, ln(P/2 + 1) - ln j) - 1/P,
 * k = 1 for the best (smallest loss) individual. */
void or_snes_utilities(int n_pop, double* u) {
  double tot = 0.0;
  for (int k = 1; k <= n_pop; ++k) {
    double v = log(n_pop / 2.0 + 1.0) - log((double)k);
    u[k - 1] = v > 0.0 ? v : 0.0;
    tot += u[k - 1];
  }
  for (int k = 0; k < n_pop; ++k) u[k] = u[k] / tot - 1.0 / n_pop;
}

/* a ranks after b: larger loss, or a NaN loss after any number. */
static int or_ranks_after(double a, double b) {
  if (isnan(a)) return !isnan(b);
  if (isnan(b)) return 0;
  return a > b;
}

/* Sort individuals by loss, smallest first (Sec. II E 2, step (b)); NaN
 * losses rank last; equal losses (and NaNs among themselves) keep index
 * order. */
void or_snes_order(int n_pop, const double* loss, int* order) {
  for (int k = 0; k < n_pop; ++k) order[k] = k;
  for (int a = 1; a < n_pop; ++a) { /* insertion sort is stable */
    int v = order[a];
    int b = a - 1;
    while (b >= 0 && or_ranks_after(loss[order[b]], loss[v])) {
      order[b + 1] = order[b];
      --b;
    }
    order[b + 1] = v;
  }
}

/* One SNES update of (m, s) from the noise r [n_pop][n_par] and the losses:
 * grad_m = sum_k u_k r_k, grad_s = sum_k u_k (r_k^2 - 1) over individuals in
 * rank order; m += eta_m s . grad_m; s *= exp(eta_s / 2 grad_s).
 * Arithmetic in float64; m and s are stored as float32. */
void or_snes_update(int n_par, int n_pop, float* m, float* s, const float* r, const double* loss,
                    double eta_m, double eta_s) {
  double u[1024];
  int order[1024];
  or_snes_utilities(n_pop, u);
  or_snes_order(n_pop, loss, order);
  for (int v = 0; v < n_par; ++v) {
    double gm = 0.0, gs = 0.0;
    for (int rank = 0; rank < n_pop; ++rank) {
      double rv = r[(size_t)order[rank] * n_par + v];
      gm += u[rank] * rv;
      gs += u[rank] * (rv * rv - 1.0);
    }
    double sv = s[v];
    m[v] = (float)((double)m[v] + eta_m * sv * gm);
    s[v] = (float)(sv * exp(0.5 * eta_s * gs));
  }
}

/* Default learning rate of the scale: (3 + ln N_par) / (5 sqrt(N_par)). */
double or_snes_eta_s(int n_par) { return (3.0 + log((double)n_par)) / (5.0 * sqrt((double)n_par)); }
