/*
 * Plain FP64 CPU reference ("the oracle") of the multilevel summation method
 * (MSM) for electrostatic energy, per-atom potentials and forces.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  The GPU product
 * path never calls it, links it or shares code with it.
 *
 * Every stage is written as the plain definition from the thesis, Sec. 2.3
 * "Multilevel Summation Method":
 *   - kernel splitting 1/r = g* + g^0 + ... + g^{l-1}        (eq. msmgrid)
 *   - Taylor smoothing gamma                                   (gamma display after eq. msmgrid)
 *   - nodal basis phi^k_mu = Phi(.)Phi(.)Phi(.)                (nodal basis display)
 *   - short range, anterpolation, restriction, lattice cutoff,
 *     top level, prolongation, interpolation                   (itemised MSM algorithm)
 *   - U_i ~ (u_i^short + u_i^long) / (4 pi eps0)               (potential display)
 *   - F_i = -dU/dr_i                                           (Sec. 2.1 "Simulation loop")
 * There is no blocking, fusion or reordering beyond those definitions: each
 * output value is one sum in a fixed order, evaluated in double precision,
 * so results do not depend on the OpenMP thread count.
 *
 * Readings taken where the thesis is silent (each is listed in the design
 * notes of the repository):
 *   - gamma of degree m is the degree-m Taylor polynomial of s^{-1/2} about
 *     s = 1 with s = rho^2 (the thesis prints m = 2);
 *   - Phi is the C1 cubic (order 4) or C1 quintic (order 6) numerical-Hermite
 *     interpolant (the thesis names only "cubic interpolating polynomial");
 *   - free-space (non-periodic) boundaries, grid origin at the box corner,
 *     level-k node mu at lo + 2^k h mu, each level spanning every node with a
 *     non-zero weight;
 *   - the self term q_i gamma(0)/a is removed from each potential;
 *   - no bonded exclusions: all pairs interact.
 *
 * Parity unpinned against the thesis (it prints nothing these readings could
 * be compared with; the test suite pins them only by mathematics and
 * invariants): the quintic basis and its pairing with m = 3, the automatic
 * level count (fewest levels whose top grid interior is at most 8 nodes per
 * side), free-space boundaries and the absence of exclusions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_LEVELS 12
#define OR_PI 3.14159265358979323846
#define OR_MAX_M 8

enum {
  OR_OK = 0,
  OR_EINVAL = -1,       /* bad parameter */
  OR_EOUTBOX = -2,      /* atom outside [lo, lo+len] */
  OR_ENONFINITE = -3,   /* NaN/Inf position or charge */
  OR_ECOINCIDENT = -7   /* two atoms at the same point (1/r undefined) */
};

typedef struct {
  double a;          /* cutoff distance of the finest level (A) */
  double h;          /* spacing of the finest grid (A) */
  int order;         /* interpolation order: 4 cubic, 6 quintic */
  int m;             /* smoothing degree (gamma is a polynomial of degree 2m); 0 -> order/2 */
  int levels;        /* number of grid levels l >= 1; 0 -> automatic */
  double lo[3];      /* box lower corner = grid origin */
  double len[3];     /* box edge lengths */
  double ke;         /* energy prefactor 1/(4 pi eps0); 0 -> 1 */
} oracle_params;

/* ------------------------------------------------------------------------- */
/* Smoothing gamma (Sec. 2.3, gamma display).                                */
/* gamma(rho) = sum_k c_k rho^{2k} for rho < 1, 1/rho for rho >= 1, with the */
/* c_k the coefficients of the degree-m Taylor polynomial of s^{-1/2} about  */
/* s = 1, re-expanded in powers of s = rho^2.  m = 2 gives 15/8, -5/4, 3/8.  */
/* ------------------------------------------------------------------------- */
static double binom_real(double x, int j) {      /* generalised binomial C(x, j) */
  double r = 1.0;
  for (int i = 0; i < j; ++i) r *= (x - i) / (i + 1);
  return r;
}

static double binom_int(int n, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r = r * (n - i) / (i + 1);
  return r;
}

void oracle_gamma_coeffs(int m, double* c /* [m+1] */) {
  for (int k = 0; k <= m; ++k) c[k] = 0.0;
  for (int j = 0; j <= m; ++j) {
    double tj = binom_real(-0.5, j);               /* Taylor coefficient of (s-1)^j */
    for (int k = 0; k <= j; ++k)                   /* (s-1)^j = sum_k C(j,k) s^k (-1)^{j-k} */
      c[k] += tj * binom_int(j, k) * (((j - k) & 1) ? -1.0 : 1.0);
  }
}

static double gamma_eval(const double* c, int m, double rho) {
  if (rho >= 1.0) return 1.0 / rho;
  double s = rho * rho, r = 0.0, p = 1.0;
  for (int k = 0; k <= m; ++k) { r += c[k] * p; p *= s; }
  return r;
}

static double dgamma_eval(const double* c, int m, double rho) {   /* d gamma / d rho */
  if (rho >= 1.0) return -1.0 / (rho * rho);
  double s = rho * rho, r = 0.0, p = rho;                           /* p = rho^{2k-1} */
  for (int k = 1; k <= m; ++k) { r += 2.0 * k * c[k] * p; p *= s; }
  return r;
}

/* ------------------------------------------------------------------------- */
/* Split kernels (eq. msmgrid).                                              */
/*   g*(r)      = 1/r - gamma(r/a)/a                                         */
/*   g^k(r)     = gamma(r/(2^k a))/(2^k a) - gamma(r/(2^{k+1} a))/(2^{k+1} a) */
/*   g^{l-1}(r) = gamma(r/(2^{l-1} a))/(2^{l-1} a)                           */
/* ------------------------------------------------------------------------- */
typedef struct {
  double a, h;
  int order, m, levels;
  double lo[3], len[3], ke;
  double c[OR_MAX_M + 1];
  int glo[OR_MAX_LEVELS][3];   /* lowest node index per level and dimension */
  int gn[OR_MAX_LEVELS][3];    /* node count per level and dimension */
  size_t goff[OR_MAX_LEVELS + 1];
} ctx_t;

static double g_short(const ctx_t* C, double r) {
  return 1.0 / r - gamma_eval(C->c, C->m, r / C->a) / C->a;
}

static double dg_short(const ctx_t* C, double r) {   /* d g* / d r */
  return -1.0 / (r * r) - dgamma_eval(C->c, C->m, r / C->a) / (C->a * C->a);
}

static double g_level(const ctx_t* C, int k, double r) {
  double ak = ldexp(C->a, k), ak1 = ldexp(C->a, k + 1);
  if (k == C->levels - 1) return gamma_eval(C->c, C->m, r / ak) / ak;
  return gamma_eval(C->c, C->m, r / ak) / ak - gamma_eval(C->c, C->m, r / ak1) / ak1;
}

/* ------------------------------------------------------------------------- */
/* One-dimensional basis Phi (nodal basis display, phi^k_mu = Phi Phi Phi).  */
/* Cubic C1 numerical Hermite (support |u| < 2):                             */
/*   (1-t)(1+t-3t^2/2) for t<=1,  -(t-1)(2-t)^2/2 for 1<=t<=2, t = |u|.       */
/* Quintic C1 (support |u| < 3):                                             */
/*   (1-t^2)(2-t)(6+3t-5t^2)/12, (1-t)(2-t)(3-t)(4+9t-5t^2)/24,              */
/*   (t-1)(t-2)(t-3)^2(4-t)/24 on [0,1], [1,2], [2,3].                        */
/* ------------------------------------------------------------------------- */
double oracle_Phi(int order, double u) {
  double t = fabs(u);
  if (order == 4) {
    if (t <= 1.0) return (1.0 - t) * (1.0 + t - 1.5 * t * t);
    if (t <= 2.0) return -0.5 * (t - 1.0) * (2.0 - t) * (2.0 - t);
    return 0.0;
  }
  if (t <= 1.0) return (1.0 - t * t) * (2.0 - t) * (6.0 + 3.0 * t - 5.0 * t * t) / 12.0;
  if (t <= 2.0) return (1.0 - t) * (2.0 - t) * (3.0 - t) * (4.0 + 9.0 * t - 5.0 * t * t) / 24.0;
  if (t <= 3.0) return (t - 1.0) * (t - 2.0) * (t - 3.0) * (t - 3.0) * (4.0 - t) / 24.0;
  return 0.0;
}

double oracle_dPhi(int order, double u) {      /* d Phi / d u, product rule on each piece */
  double t = fabs(u), sg = (u < 0.0) ? -1.0 : 1.0, d;
  if (order == 4) {
    if (t <= 1.0) d = -(1.0 + t - 1.5 * t * t) + (1.0 - t) * (1.0 - 3.0 * t);
    else if (t <= 2.0) d = -0.5 * ((2.0 - t) * (2.0 - t) - 2.0 * (t - 1.0) * (2.0 - t));
    else d = 0.0;
    return sg * d;
  }
  if (t <= 1.0) {
    double A = 1.0 - t * t, B = 2.0 - t, Cc = 6.0 + 3.0 * t - 5.0 * t * t;
    d = (-2.0 * t * B * Cc - A * Cc + A * B * (3.0 - 10.0 * t)) / 12.0;
  } else if (t <= 2.0) {
    double A = 1.0 - t, B = 2.0 - t, Cc = 3.0 - t, D = 4.0 + 9.0 * t - 5.0 * t * t;
    d = (-B * Cc * D - A * Cc * D - A * B * D + A * B * Cc * (9.0 - 10.0 * t)) / 24.0;
  } else if (t <= 3.0) {
    double A = t - 1.0, B = t - 2.0, Cc = (t - 3.0) * (t - 3.0), D = 4.0 - t;
    d = (B * Cc * D + A * Cc * D + A * B * 2.0 * (t - 3.0) * D - A * B * Cc) / 24.0;
  } else {
    d = 0.0;
  }
  return sg * d;
}

/* ------------------------------------------------------------------------- */
/* Grid hierarchy.  Level k has spacing 2^k h (eq. msmgrid: level k carries   */
/* cutoff 2^k a; nodal basis display: spacing 2^k h).  Node mu of level k     */
/* sits at lo + 2^k h mu.  Level 0 spans every node an atom in the box       */
/* touches; level k+1 spans every coarse node a level-k node restricts to.   */
/* ------------------------------------------------------------------------- */
static int floordiv2(int v) { return (v >= 0) ? v / 2 : -((-v + 1) / 2); }
static int ceildiv2(int v) { return -floordiv2(-v); }

static int auto_levels(double maxlen, double h) {
  for (int l = 1; l <= OR_MAX_LEVELS; ++l)
    if ((int)ceil(maxlen / ldexp(h, l - 1)) + 1 <= 8) return l;
  return OR_MAX_LEVELS;
}

static int ctx_init(ctx_t* C, const oracle_params* p) {
  memset(C, 0, sizeof(*C));
  if (!(p->a > 0.0) || !(p->h > 0.0) || !isfinite(p->a) || !isfinite(p->h)) return OR_EINVAL;
  if (p->order != 4 && p->order != 6) return OR_EINVAL;
  C->a = p->a; C->h = p->h; C->order = p->order;
  C->m = p->m ? p->m : p->order / 2;
  if (C->m < 1 || C->m > OR_MAX_M) return OR_EINVAL;
  C->ke = (p->ke != 0.0) ? p->ke : 1.0;
  double maxlen = 0.0;
  for (int d = 0; d < 3; ++d) {
    if (!(p->len[d] > 0.0) || !isfinite(p->len[d]) || !isfinite(p->lo[d])) return OR_EINVAL;
    C->lo[d] = p->lo[d]; C->len[d] = p->len[d];
    if (p->len[d] > maxlen) maxlen = p->len[d];
  }
  C->levels = p->levels ? p->levels : auto_levels(maxlen, p->h);
  if (C->levels < 1 || C->levels > OR_MAX_LEVELS) return OR_EINVAL;
  oracle_gamma_coeffs(C->m, C->c);
  int half = C->order / 2;
  C->goff[0] = 0;
  for (int k = 0; k < C->levels; ++k) {
    for (int d = 0; d < 3; ++d) {
      int lo, hi;
      if (k == 0) {
        lo = -(half - 1);
        hi = (int)floor(C->len[d] / C->h) + half;
      } else {
        int plo = C->glo[k - 1][d], phi = plo + C->gn[k - 1][d] - 1;
        lo = ceildiv2(plo - (C->order - 1));
        hi = floordiv2(phi + (C->order - 1));
      }
      C->glo[k][d] = lo;
      C->gn[k][d] = hi - lo + 1;
    }
    C->goff[k + 1] = C->goff[k] + (size_t)C->gn[k][0] * C->gn[k][1] * C->gn[k][2];
  }
  return OR_OK;
}

static size_t gidx(const ctx_t* C, int k, int ix, int iy, int iz) {
  return C->goff[k] + ((size_t)(iz - C->glo[k][2]) * C->gn[k][1] + (size_t)(iy - C->glo[k][1])) *
                          C->gn[k][0] + (size_t)(ix - C->glo[k][0]);
}

/* Public: level count and per-level node ranges (lo index and count per dim). */
int oracle_layout(const oracle_params* p, int* levels, int* glo /* [L][3] */, int* gn /* [L][3] */) {
  ctx_t C;
  int rc = ctx_init(&C, p);
  if (rc) return rc;
  *levels = C.levels;
  for (int k = 0; k < C.levels; ++k)
    for (int d = 0; d < 3; ++d) { glo[3 * k + d] = C.glo[k][d]; gn[3 * k + d] = C.gn[k][d]; }
  return OR_OK;
}

double oracle_gamma(int m, double rho) {
  double c[OR_MAX_M + 1];
  oracle_gamma_coeffs(m, c);
  return gamma_eval(c, m, rho);
}

double oracle_dgamma(int m, double rho) {
  double c[OR_MAX_M + 1];
  oracle_gamma_coeffs(m, c);
  return dgamma_eval(c, m, rho);
}

/* g* (k = -1), g^k (0 <= k < levels); exposed for the splitting identity check */
double oracle_split_kernel(const oracle_params* p, int k, double r) {
  ctx_t C;
  if (ctx_init(&C, p)) return NAN;
  if (k < 0) return g_short(&C, r);
  return g_level(&C, k, r);
}

/* ------------------------------------------------------------------------- */
/* Input validation: finite values, every atom inside [lo, lo + len].         */
/* ------------------------------------------------------------------------- */
static int check_atoms(const ctx_t* C, int n, const double* x, const double* y, const double* z,
                       const double* q) {
  const double* r[3] = {x, y, z};
  for (int i = 0; i < n; ++i) {
    if (!isfinite(q[i])) return OR_ENONFINITE;
    for (int d = 0; d < 3; ++d)
      if (!isfinite(r[d][i])) return OR_ENONFINITE;
  }
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d)
      if (r[d][i] < C->lo[d] || r[d][i] > C->lo[d] + C->len[d]) return OR_EOUTBOX;
  return OR_OK;
}

/* Neumaier-compensated running sum */
typedef struct { double s, c; } nsum_t;
static void nsum_add(nsum_t* a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
  else a->c += (v - t) + a->s;
  a->s = t;
}

/* ------------------------------------------------------------------------- */
/* Short-range part: u_i^short = sum_j g*(r_i, r_j) q_j over j with          */
/* |r_i - r_j| < a (itemised algorithm, short-range sentence), found through */
/* link cells of edge >= a (Sec. 2.1 "Potentials", link-cell method).        */
/* Force: F_i^short = -q_i sum_j q_j g*'(r_ij) (r_i - r_j)/r_ij.             */
/* mode 0: link cells; mode 1: every pair (brute force).                     */
/* ------------------------------------------------------------------------- */
static int short_range(const ctx_t* C, int n, const double* x, const double* y, const double* z,
                       const double* q, const int* sample, int ns, int mode, double* phis,
                       double* fsx, double* fsy, double* fsz) {
  int nc[3];
  double cs[3];
  for (int d = 0; d < 3; ++d) {
    nc[d] = (int)floor(C->len[d] / C->a);
    if (nc[d] < 1) nc[d] = 1;
    cs[d] = C->len[d] / nc[d];
  }
  size_t ncell = (size_t)nc[0] * nc[1] * nc[2];
  int* cell = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int* start = (int*)calloc(ncell + 1, sizeof(int));
  int* list = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  const double* r[3] = {x, y, z};
  for (int i = 0; i < n; ++i) {
    int c3[3];
    for (int d = 0; d < 3; ++d) {
      int c = (int)floor((r[d][i] - C->lo[d]) / cs[d]);
      c3[d] = c < 0 ? 0 : (c >= nc[d] ? nc[d] - 1 : c);
    }
    cell[i] = (c3[2] * nc[1] + c3[1]) * nc[0] + c3[0];
    start[cell[i] + 1]++;
  }
  for (size_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
  {
    int* fill = (int*)malloc(sizeof(int) * ncell);
    for (size_t c = 0; c < ncell; ++c) fill[c] = start[c];
    for (int i = 0; i < n; ++i) list[fill[cell[i]]++] = i;   /* stable: increasing i per cell */
    free(fill);
  }
  const double a2 = C->a * C->a;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
  for (int s = 0; s < ns; ++s) {
    int i = sample ? sample[s] : s;
    double ps = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    if (mode == 1) {
      for (int j = 0; j < n; ++j) {
        if (j == i) continue;
        double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= a2) continue;
        if (r2 == 0.0) { bad = 1; continue; }
        double rr = sqrt(r2);
        ps += q[j] * g_short(C, rr);
        double w = -q[i] * q[j] * dg_short(C, rr) / rr;
        fx += w * dx; fy += w * dy; fz += w * dz;
      }
    } else {
      int ci = cell[i], cx = ci % nc[0], cy = (ci / nc[0]) % nc[1], cz = ci / (nc[0] * nc[1]);
      for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
          for (int ox = -1; ox <= 1; ++ox) {
            int jx = cx + ox, jy = cy + oy, jz = cz + oz;
            if (jx < 0 || jy < 0 || jz < 0 || jx >= nc[0] || jy >= nc[1] || jz >= nc[2]) continue;
            int cj = (jz * nc[1] + jy) * nc[0] + jx;
            for (int t = start[cj]; t < start[cj + 1]; ++t) {
              int j = list[t];
              if (j == i) continue;
              double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
              double r2 = dx * dx + dy * dy + dz * dz;
              if (r2 >= a2) continue;
              if (r2 == 0.0) { bad = 1; continue; }
              double rr = sqrt(r2);
              ps += q[j] * g_short(C, rr);
              double w = -q[i] * q[j] * dg_short(C, rr) / rr;
              fx += w * dx; fy += w * dy; fz += w * dz;
            }
          }
    }
    phis[i] = ps; fsx[i] = fx; fsy[i] = fy; fsz[i] = fz;
  }
  free(cell); free(start); free(list);
  return bad ? OR_ECOINCIDENT : OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Anterpolation: q^0_mu = sum_j phi^0_mu(r_j) q_j (itemised algorithm).     */
/* phi^0_mu(r) = Phi((x - x_mu)/h) Phi((y - y_mu)/h) Phi((z - z_mu)/h); only */
/* nodes floor(t) - (order/2 - 1) .. floor(t) + order/2 can be non-zero.     */
/* Serial scatter in atom order, so the sum order is fixed.                  */
/* ------------------------------------------------------------------------- */
static void anterpolate(const ctx_t* C, int n, const double* x, const double* y, const double* z,
                        const double* q, double* grid) {
  const double* r[3] = {x, y, z};
  int half = C->order / 2, no = C->order;
  for (int i = 0; i < n; ++i) {
    double t[3], w[3][8];
    int f[3];
    for (int d = 0; d < 3; ++d) {
      t[d] = (r[d][i] - C->lo[d]) / C->h;
      f[d] = (int)floor(t[d]);
      for (int s = 0; s < no; ++s) w[d][s] = oracle_Phi(C->order, t[d] - (f[d] - (half - 1) + s));
    }
    for (int sz = 0; sz < no; ++sz)
      for (int sy = 0; sy < no; ++sy)
        for (int sx = 0; sx < no; ++sx)
          grid[gidx(C, 0, f[0] - (half - 1) + sx, f[1] - (half - 1) + sy, f[2] - (half - 1) + sz)] +=
              q[i] * w[0][sx] * w[1][sy] * w[2][sz];
  }
}

/* ------------------------------------------------------------------------- */
/* Restriction: q^{k+1}_mu = sum_nu phi^{k+1}_mu(r^k_nu) q^k_nu              */
/* (itemised algorithm).  With r^k_nu = lo + 2^k h nu and r^{k+1}_mu =       */
/* lo + 2^{k+1} h mu, the basis argument is nu/2 - mu per dimension; it is   */
/* non-zero only for |nu - 2 mu| <= order - 1.                               */
/* ------------------------------------------------------------------------- */
static void restrict_level(const ctx_t* C, int k, const double* grid_in, double* grid_out) {
  int R = C->order - 1;
  const int* lo = C->glo[k + 1];
  const int* gn = C->gn[k + 1];
  const int* flo = C->glo[k];
  const int* fn = C->gn[k];
#pragma omp parallel for collapse(2) schedule(static)
  for (int mz = lo[2]; mz < lo[2] + gn[2]; ++mz)
    for (int my = lo[1]; my < lo[1] + gn[1]; ++my)
      for (int mx = lo[0]; mx < lo[0] + gn[0]; ++mx) {
        double s = 0.0;
        for (int vz = 2 * mz - R; vz <= 2 * mz + R; ++vz) {
          if (vz < flo[2] || vz >= flo[2] + fn[2]) continue;
          double wz = oracle_Phi(C->order, 0.5 * vz - mz);
          for (int vy = 2 * my - R; vy <= 2 * my + R; ++vy) {
            if (vy < flo[1] || vy >= flo[1] + fn[1]) continue;
            double wy = oracle_Phi(C->order, 0.5 * vy - my);
            for (int vx = 2 * mx - R; vx <= 2 * mx + R; ++vx) {
              if (vx < flo[0] || vx >= flo[0] + fn[0]) continue;
              double wx = oracle_Phi(C->order, 0.5 * vx - mx);
              s += wx * wy * wz * grid_in[gidx(C, k, vx, vy, vz)];
            }
          }
        }
        grid_out[gidx(C, k + 1, mx, my, mz)] = s;
      }
}

/* ------------------------------------------------------------------------- */
/* Lattice cutoff (k <= l-2) and top level (k = l-1):                        */
/*   u^{k}_mu = sum_nu g^k(r^k_mu, r^k_nu) q^k_nu                            */
/* with |r^k_mu - r^k_nu| = 2^k h |mu - nu|.  Below the top g^k vanishes for */
/* distances >= 2^{k+1} a, so only |mu - nu| < 2a/h contributes; the top     */
/* level sums over every node.  `need` (nullable) restricts the outputs to   */
/* flagged nodes; each output is still the full sum.                         */
/* ------------------------------------------------------------------------- */
static void lattice_level(const ctx_t* C, int k, const double* qk, double* uk, const uint8_t* need) {
  const int* lo = C->glo[k];
  const int* gn = C->gn[k];
  const int top = (k == C->levels - 1);
  const double hk = ldexp(C->h, k);
  const double rcut = ldexp(C->a, k + 1);
  const int R = top ? (gn[0] > gn[1] ? (gn[0] > gn[2] ? gn[0] : gn[2]) : (gn[1] > gn[2] ? gn[1] : gn[2]))
                    : (int)ceil(2.0 * C->a / C->h);
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int mz = lo[2]; mz < lo[2] + gn[2]; ++mz)
    for (int my = lo[1]; my < lo[1] + gn[1]; ++my)
      for (int mx = lo[0]; mx < lo[0] + gn[0]; ++mx) {
        size_t om = gidx(C, k, mx, my, mz);
        if (need && !need[om]) continue;
        double s = 0.0;
        for (int vz = mz - R; vz <= mz + R; ++vz) {
          if (vz < lo[2] || vz >= lo[2] + gn[2]) continue;
          for (int vy = my - R; vy <= my + R; ++vy) {
            if (vy < lo[1] || vy >= lo[1] + gn[1]) continue;
            for (int vx = mx - R; vx <= mx + R; ++vx) {
              if (vx < lo[0] || vx >= lo[0] + gn[0]) continue;
              double dx = (double)(mx - vx), dy = (double)(my - vy), dz = (double)(mz - vz);
              double d = hk * sqrt(dx * dx + dy * dy + dz * dz);
              if (!top && d >= rcut) continue;
              s += g_level(C, k, d) * qk[gidx(C, k, vx, vy, vz)];
            }
          }
        }
        uk[om] = s;
      }
}

/* ------------------------------------------------------------------------- */
/* Prolongation: u^k_mu = u^{k,cutoff}_mu + sum_nu phi^{k+1}_nu(r^k_mu)       */
/* u^{k+1}_nu (itemised algorithm); the basis argument is mu/2 - nu.          */
/* ------------------------------------------------------------------------- */
static void prolong_level(const ctx_t* C, int k, const double* ucoarse, double* ufine, const uint8_t* need) {
  int R = C->order - 1;
  const int* lo = C->glo[k];
  const int* gn = C->gn[k];
  const int* clo = C->glo[k + 1];
  const int* cn = C->gn[k + 1];
#pragma omp parallel for collapse(2) schedule(static)
  for (int mz = lo[2]; mz < lo[2] + gn[2]; ++mz)
    for (int my = lo[1]; my < lo[1] + gn[1]; ++my)
      for (int mx = lo[0]; mx < lo[0] + gn[0]; ++mx) {
        size_t om = gidx(C, k, mx, my, mz);
        if (need && !need[om]) continue;
        double s = 0.0;
        for (int vz = clo[2]; vz < clo[2] + cn[2]; ++vz) {
          if (abs(mz - 2 * vz) > R) continue;
          double wz = oracle_Phi(C->order, 0.5 * mz - vz);
          for (int vy = clo[1]; vy < clo[1] + cn[1]; ++vy) {
            if (abs(my - 2 * vy) > R) continue;
            double wy = oracle_Phi(C->order, 0.5 * my - vy);
            for (int vx = clo[0]; vx < clo[0] + cn[0]; ++vx) {
              if (abs(mx - 2 * vx) > R) continue;
              double wx = oracle_Phi(C->order, 0.5 * mx - vx);
              s += wx * wy * wz * ucoarse[gidx(C, k + 1, vx, vy, vz)];
            }
          }
        }
        ufine[om] += s;
      }
}

/* ------------------------------------------------------------------------- */
/* Interpolation: u_i^long = sum_mu phi^0_mu(r_i) u^0_mu and its gradient    */
/* (itemised algorithm), the gradient of the basis by the product rule.      */
/* ------------------------------------------------------------------------- */
static void interpolate(const ctx_t* C, const double* x, const double* y, const double* z,
                        const int* sample, int ns, const double* u0, double* phil, double* gx,
                        double* gy, double* gz) {
  const double* r[3] = {x, y, z};
  int half = C->order / 2, no = C->order;
#pragma omp parallel for schedule(static)
  for (int s = 0; s < ns; ++s) {
    int i = sample ? sample[s] : s;
    double t[3], w[3][8], dw[3][8];
    int f[3];
    for (int d = 0; d < 3; ++d) {
      t[d] = (r[d][i] - C->lo[d]) / C->h;
      f[d] = (int)floor(t[d]);
      for (int e = 0; e < no; ++e) {
        double u = t[d] - (f[d] - (half - 1) + e);
        w[d][e] = oracle_Phi(C->order, u);
        dw[d][e] = oracle_dPhi(C->order, u) / C->h;
      }
    }
    double p = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    for (int sz = 0; sz < no; ++sz)
      for (int sy = 0; sy < no; ++sy)
        for (int sx = 0; sx < no; ++sx) {
          double u = u0[gidx(C, 0, f[0] - (half - 1) + sx, f[1] - (half - 1) + sy, f[2] - (half - 1) + sz)];
          p += w[0][sx] * w[1][sy] * w[2][sz] * u;
          ax += dw[0][sx] * w[1][sy] * w[2][sz] * u;
          ay += w[0][sx] * dw[1][sy] * w[2][sz] * u;
          az += w[0][sx] * w[1][sy] * dw[2][sz] * u;
        }
    phil[i] = p; gx[i] = ax; gy[i] = ay; gz[i] = az;
  }
}

/* Mark the level-0 nodes that sampled atoms read, then the coarse nodes that  */
/* prolongation reads for each marked fine node.                               */
static void mark_needed(const ctx_t* C, const double* x, const double* y, const double* z,
                        const int* sample, int ns, uint8_t* need) {
  const double* r[3] = {x, y, z};
  int half = C->order / 2, no = C->order, R = C->order - 1;
  for (int s = 0; s < ns; ++s) {
    int i = sample[s], f[3];
    for (int d = 0; d < 3; ++d) f[d] = (int)floor((r[d][i] - C->lo[d]) / C->h);
    for (int sz = 0; sz < no; ++sz)
      for (int sy = 0; sy < no; ++sy)
        for (int sx = 0; sx < no; ++sx)
          need[gidx(C, 0, f[0] - (half - 1) + sx, f[1] - (half - 1) + sy, f[2] - (half - 1) + sz)] = 1;
  }
  for (int k = 0; k + 1 < C->levels; ++k) {
    const int* lo = C->glo[k];
    const int* gn = C->gn[k];
    const int* clo = C->glo[k + 1];
    const int* cn = C->gn[k + 1];
    for (int mz = lo[2]; mz < lo[2] + gn[2]; ++mz)
      for (int my = lo[1]; my < lo[1] + gn[1]; ++my)
        for (int mx = lo[0]; mx < lo[0] + gn[0]; ++mx) {
          if (!need[gidx(C, k, mx, my, mz)]) continue;
          for (int vz = clo[2]; vz < clo[2] + cn[2]; ++vz) {
            if (abs(mz - 2 * vz) > R) continue;
            for (int vy = clo[1]; vy < clo[1] + cn[1]; ++vy) {
              if (abs(my - 2 * vy) > R) continue;
              for (int vx = clo[0]; vx < clo[0] + cn[0]; ++vx) {
                if (abs(mx - 2 * vx) > R) continue;
                need[gidx(C, k + 1, vx, vy, vz)] = 1;
              }
            }
          }
        }
  }
}

/* ------------------------------------------------------------------------- */
/* Full evaluation.                                                          */
/*   phi_i = ke (u_i^short + u_i^long - q_i gamma(0)/a)                      */
/*   E     = 1/2 sum_i q_i phi_i                                             */
/*   F_i   = ke (F_i^short - q_i grad u_i^long)                               */
/*   W_ab  = sum_i (r_i - lo)_a F_i,b                                         */
/* Inputs: n atoms, positions x,y,z and charges q (float64, host).           */
/* Outputs (all nullable): fx,fy,fz,phi [n]; energy [1]; virial [9];         */
/*   qgrid, ucut, ugrid: concatenated level grids (oracle_layout order,      */
/*   x fastest): grid charges q^k, lattice-cutoff / top-level sums u^{k,cut}, */
/*   and the prolongated potentials u^k; phis [n]: short-range potential.    */
/* sample (nullable): evaluate only these atoms' outputs; energy and virial  */
/*   are then not written.  short_mode: 0 link cells, 1 all pairs.           */
/* Returns 0 or a negative error code.                                       */
/* ------------------------------------------------------------------------- */
int oracle_msm(const oracle_params* p, int n, const double* x, const double* y, const double* z,
               const double* q, double* fx, double* fy, double* fz, double* phi, double* energy,
               double* virial, double* qgrid, double* ucut, double* ugrid, double* phis_out,
               const int* sample, int ns, int short_mode, int nthreads) {
  ctx_t C;
  int rc = ctx_init(&C, p);
  if (rc) return rc;
  if (n < 0) return OR_EINVAL;
  if (n > 0 && (!x || !y || !z || !q)) return OR_EINVAL;
  rc = check_atoms(&C, n, x, y, z, q);
  if (rc) return rc;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  if (!sample) ns = n;
  for (int s = 0; sample && s < ns; ++s)
    if (sample[s] < 0 || sample[s] >= n) return OR_EINVAL;

  size_t ng = C.goff[C.levels];
  double* qg = (double*)calloc(ng, sizeof(double));
  double* uc = (double*)calloc(ng, sizeof(double));
  double* ug = (double*)calloc(ng, sizeof(double));
  size_t na = (size_t)(n > 0 ? n : 1);
  double* ps = (double*)calloc(na, sizeof(double));
  double* fsx = (double*)calloc(na, sizeof(double));
  double* fsy = (double*)calloc(na, sizeof(double));
  double* fsz = (double*)calloc(na, sizeof(double));
  double* pl = (double*)calloc(na, sizeof(double));
  double* gx = (double*)calloc(na, sizeof(double));
  double* gy = (double*)calloc(na, sizeof(double));
  double* gz = (double*)calloc(na, sizeof(double));
  uint8_t* need = NULL;

  rc = short_range(&C, n, x, y, z, q, sample, ns, short_mode, ps, fsx, fsy, fsz);
  if (rc) goto done;

  if (sample) {
    need = (uint8_t*)calloc(ng, 1);
    mark_needed(&C, x, y, z, sample, ns, need);
  }

  anterpolate(&C, n, x, y, z, q, qg);
  for (int k = 0; k + 1 < C.levels; ++k) restrict_level(&C, k, qg, qg);
  for (int k = 0; k < C.levels; ++k) lattice_level(&C, k, qg, uc, need);
  memcpy(ug, uc, ng * sizeof(double));
  for (int k = C.levels - 2; k >= 0; --k) prolong_level(&C, k, ug, ug, need);
  interpolate(&C, x, y, z, sample, ns, ug, pl, gx, gy, gz);

  {
    const double self = gamma_eval(C.c, C.m, 0.0) / C.a;     /* gamma(0)/a */
    nsum_t e = {0.0, 0.0};
    nsum_t w[9];
    memset(w, 0, sizeof(w));
    for (int s = 0; s < ns; ++s) {
      int i = sample ? sample[s] : s;
      double ph = C.ke * (ps[i] + pl[i] - q[i] * self);
      double f3[3] = {C.ke * (fsx[i] - q[i] * gx[i]), C.ke * (fsy[i] - q[i] * gy[i]),
                      C.ke * (fsz[i] - q[i] * gz[i])};
      double r3[3] = {x[i] - C.lo[0], y[i] - C.lo[1], z[i] - C.lo[2]};
      if (phi) phi[i] = ph;
      if (fx) fx[i] = f3[0];
      if (fy) fy[i] = f3[1];
      if (fz) fz[i] = f3[2];
      if (phis_out) phis_out[i] = C.ke * ps[i];
      nsum_add(&e, 0.5 * q[i] * ph);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) nsum_add(&w[3 * a + b], r3[a] * f3[b]);
    }
    if (!sample) {
      if (energy) *energy = e.s + e.c;
      if (virial)
        for (int t = 0; t < 9; ++t) virial[t] = w[t].s + w[t].c;
    }
  }
  if (qgrid) memcpy(qgrid, qg, ng * sizeof(double));
  if (ucut) memcpy(ucut, uc, ng * sizeof(double));
  if (ugrid) memcpy(ugrid, ug, ng * sizeof(double));

done:
  free(qg); free(uc); free(ug); free(ps); free(fsx); free(fsy); free(fsz);
  free(pl); free(gx); free(gy); free(gz); free(need);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Direct Coulomb sum (eq. coulomb), each unordered pair once, no self term: */
/*   E = sum_{i<j} q_i q_j / r_ij,  phi_i = sum_{j != i} q_j / r_ij,         */
/*   F_i = sum_{j != i} q_i q_j (r_i - r_j) / r_ij^3.  Times ke.             */
/* The exact target the multilevel approximation is measured against.       */
/* ------------------------------------------------------------------------- */
int oracle_direct(int n, const double* x, const double* y, const double* z, const double* q,
                  double ke, double* fx, double* fy, double* fz, double* phi, double* energy,
                  int nthreads) {
  if (ke == 0.0) ke = 1.0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  double* ph = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
  for (int i = 0; i < n; ++i) {
    double p = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
      double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 == 0.0) { bad = 1; continue; }
      double r = sqrt(r2);
      p += q[j] / r;
      double w = q[i] * q[j] / (r2 * r);
      ax += w * dx; ay += w * dy; az += w * dz;
    }
    ph[i] = ke * p;
    if (fx) fx[i] = ke * ax;
    if (fy) fy[i] = ke * ay;
    if (fz) fz[i] = ke * az;
  }
  nsum_t e = {0.0, 0.0};
  for (int i = 0; i < n; ++i) nsum_add(&e, 0.5 * q[i] * ph[i]);
  if (phi) memcpy(phi, ph, sizeof(double) * (size_t)n);
  if (energy) *energy = e.s + e.c;
  free(ph);
  return bad ? OR_ECOINCIDENT : OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Cheap pair methods the thesis proposes as coarse propagators G (Sec. 3.2  */
/* "Proposed Solutions": "Cutoff Method", "Wolf Summation Method"; the       */
/* smoothed cutoff is named in Sec. 2.2).  Each sums a pair energy           */
/* q_i q_j e(r) over the unordered pairs closer than rc, plus a self term    */
/* s q_i^2 per atom:                                                         */
/*   kind 1, plain cutoff:  e(r) = 1/r                                       */
/*   kind 2, smoothed cutoff (shifted force; reading of the thesis, which    */
/*           names the method only): e(r) = 1/r - 1/rc + (r - rc)/rc^2,     */
/*           so e and e' vanish at rc                                        */
/*   kind 3, Wolf summation: e(r) = erfc(alpha r)/r - erfc(alpha rc)/rc,     */
/*           s = -(erfc(alpha rc)/(2 rc) + alpha/sqrt(pi))                   */
/* Outputs (times ke): E = sum_{i<j} q_i q_j e(r_ij) + s sum_i q_i^2,        */
/*   phi_i = dE/dq_i = sum_{j != i} q_j e(r_ij) + 2 s q_i,                   */
/*   F_i = -dE/dr_i = -q_i sum_{j != i} q_j e'(r_ij) (r_i - r_j)/r_ij,       */
/*   W_ab = sum_i (r_i - lo)_a F_i,b.                                        */
/* Pairs are found through cells of edge >= rc (each atom scans the 27       */
/* cells around its own), or over all pairs when all_pairs is set.  Whether  */
/* a pair is inside the cutoff is a discrete decision; with f32_cut set it is */
/* taken in float32 the way a float32 kernel takes it (differences of the    */
/* float32 coordinates, r^2 = fma(dx, dx, fma(dy, dy, dz dz)) compared with  */
/* float32(rc^2)), so both sides include the same pairs; the pair terms are  */
/* still evaluated in double.                                                */
/* ------------------------------------------------------------------------- */
static double pair_e(int kind, double rc, double alpha, double r) {
  if (kind == 1) return 1.0 / r;
  if (kind == 2) return 1.0 / r - 1.0 / rc + (r - rc) / (rc * rc);
  return erfc(alpha * r) / r - erfc(alpha * rc) / rc;
}

static double pair_de(int kind, double rc, double alpha, double r) {   /* d e / d r */
  if (kind == 1) return -1.0 / (r * r);
  if (kind == 2) return -1.0 / (r * r) + 1.0 / (rc * rc);
  return -erfc(alpha * r) / (r * r) - 2.0 * alpha / sqrt(OR_PI) * exp(-alpha * alpha * r * r) / r;
}

double oracle_pair_e(int kind, double rc, double alpha, double r) { return pair_e(kind, rc, alpha, r); }

/* For each of n pairs (a_k, b_k): whether 0 < r^2 < rc^2 holds when decided  */
/* in float32 the way a float32 kernel decides it (see f32_cut above).       */
void oracle_inside_f32(int n, const double* ax, const double* ay, const double* az, const double* bx,
                       const double* by, const double* bz, double rc, int* inside) {
  const float rc2f = (float)(rc * rc);
  for (int k = 0; k < n; ++k) {
    const float dxf = (float)ax[k] - (float)bx[k], dyf = (float)ay[k] - (float)by[k];
    const float dzf = (float)az[k] - (float)bz[k];
    const float r2f = fmaf(dxf, dxf, fmaf(dyf, dyf, dzf * dzf));
    inside[k] = (r2f > 0.0f && r2f < rc2f) ? 1 : 0;
  }
}

int oracle_pair(int kind, double rc, double alpha, const double* lo, const double* len, double ke,
                int n, const double* x, const double* y, const double* z, const double* q,
                double* fx, double* fy, double* fz, double* phi, double* energy, double* virial,
                int all_pairs, int f32_cut, int nthreads) {
  if (kind < 1 || kind > 3 || !(rc > 0.0) || !(alpha >= 0.0) || n < 0) return OR_EINVAL;
  if (ke == 0.0) ke = 1.0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  for (int d = 0; d < 3; ++d)
    if (!(len[d] > 0.0)) return OR_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i]) || !isfinite(q[i])) return OR_ENONFINITE;
    const double p3[3] = {x[i], y[i], z[i]};
    for (int d = 0; d < 3; ++d)
      if (p3[d] < lo[d] || p3[d] > lo[d] + len[d]) return OR_EOUTBOX;
  }
  const double self = (kind == 3) ? -(erfc(alpha * rc) / (2.0 * rc) + alpha / sqrt(OR_PI)) : 0.0;
  int nc[3];
  double cs[3];
  for (int d = 0; d < 3; ++d) {
    nc[d] = (int)floor(len[d] / rc);
    if (nc[d] < 1) nc[d] = 1;
    cs[d] = len[d] / nc[d];
  }
  size_t ncell = (size_t)nc[0] * nc[1] * nc[2];
  int* cell = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int* start = (int*)calloc(ncell + 1, sizeof(int));
  int* list = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  const double* r[3] = {x, y, z};
  for (int i = 0; i < n; ++i) {
    int c3[3];
    for (int d = 0; d < 3; ++d) {
      int c = (int)floor((r[d][i] - lo[d]) / cs[d]);
      c3[d] = c < 0 ? 0 : (c >= nc[d] ? nc[d] - 1 : c);
    }
    cell[i] = (c3[2] * nc[1] + c3[1]) * nc[0] + c3[0];
    start[cell[i] + 1]++;
  }
  for (size_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
  {
    int* fill = (int*)malloc(sizeof(int) * (ncell > 0 ? ncell : 1));
    for (size_t c = 0; c < ncell; ++c) fill[c] = start[c];
    for (int i = 0; i < n; ++i) list[fill[cell[i]]++] = i;
    free(fill);
  }
  double* ph = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* f3 = (double*)calloc(3 * (size_t)(n > 0 ? n : 1), sizeof(double));
  const double rc2 = rc * rc;
  const float rc2f = (float)(rc * rc);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
  for (int i = 0; i < n; ++i) {
    double p = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    int ci = cell[i], cx = ci % nc[0], cy = (ci / nc[0]) % nc[1], cz = ci / (nc[0] * nc[1]);
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          if (all_pairs && (ox || oy || oz)) continue;
          int jx = cx + ox, jy = cy + oy, jz = cz + oz;
          if (jx < 0 || jy < 0 || jz < 0 || jx >= nc[0] || jy >= nc[1] || jz >= nc[2]) continue;
          int cj = (jz * nc[1] + jy) * nc[0] + jx;
          const int t0 = all_pairs ? 0 : start[cj], t1 = all_pairs ? n : start[cj + 1];
          for (int t = t0; t < t1; ++t) {
            int j = all_pairs ? t : list[t];
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) { bad = 1; continue; }
            if (f32_cut) {
              const float dxf = (float)x[i] - (float)x[j], dyf = (float)y[i] - (float)y[j];
              const float dzf = (float)z[i] - (float)z[j];
              const float r2f = fmaf(dxf, dxf, fmaf(dyf, dyf, dzf * dzf));
              if (!(r2f > 0.0f && r2f < rc2f)) continue;
            } else if (r2 >= rc2) {
              continue;
            }
            double rr = sqrt(r2);
            p += q[j] * pair_e(kind, rc, alpha, rr);
            double w = -q[i] * q[j] * pair_de(kind, rc, alpha, rr) / rr;
            ax += w * dx; ay += w * dy; az += w * dz;
          }
        }
    ph[i] = ke * (p + 2.0 * self * q[i]);
    f3[3 * (size_t)i] = ke * ax;
    f3[3 * (size_t)i + 1] = ke * ay;
    f3[3 * (size_t)i + 2] = ke * az;
  }
  nsum_t e = {0.0, 0.0};
  nsum_t w[9];
  memset(w, 0, sizeof(w));
  for (int i = 0; i < n; ++i) {
    const double* fi = f3 + 3 * (size_t)i;
    const double r3[3] = {x[i] - lo[0], y[i] - lo[1], z[i] - lo[2]};
    nsum_add(&e, 0.5 * q[i] * ph[i]);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) nsum_add(&w[3 * a + b], r3[a] * fi[b]);
    if (fx) fx[i] = fi[0];
    if (fy) fy[i] = fi[1];
    if (fz) fz[i] = fi[2];
  }
  if (phi) memcpy(phi, ph, sizeof(double) * (size_t)n);
  if (energy) *energy = e.s + e.c;
  if (virial)
    for (int t = 0; t < 9; ++t) virial[t] = w[t].s + w[t].c;
  free(cell); free(start); free(list); free(ph); free(f3);
  return bad ? OR_ECOINCIDENT : OR_OK;
}

/* ========================================================================= */
/* Periodic boundaries.                                                      */
/* Reading (the thesis evaluates free-space systems and names periodicity    */
/* only with the Fourier methods): the box is the unit cell of an infinite   */
/* lattice of copies with periods len[d], and every sum of the method runs   */
/* over the atoms of the central box and all their images:                   */
/*   - short range: pairs (i, j, p) with |r_i - r_j + P p| < a, P = diag(len);*/
/*     2a <= len[d], so at most one image of a pair is that close;           */
/*   - level k is a periodic grid of n_k = (len / h) / 2^k nodes per         */
/*     dimension (len / h an integer divisible by 2^(l-1)); anterpolation,   */
/*     restriction, prolongation and interpolation take node indices modulo  */
/*     n_k, and the lattice cutoff sums g^k over every image of a node pair;  */
/*   - top level: K(r) = sum_p g^{l-1}(|r + P p|).  g^{l-1} decays as 1/r, so */
/*     the lattice sum is taken in the Ewald convention (conducting boundary,*/
/*     uniform neutralising background):                                     */
/*       K(r) = Psi(r) - sum_p [1/|r + P p| - g^{l-1}(|r + P p|)],          */
/*     Psi the Ewald lattice sum of 1/r; the bracket vanishes beyond         */
/*     2^{l-1} a, where gamma(rho) = 1/rho.                                  */
/* Atoms may lie anywhere; each is first mapped into [lo, lo + len).         */
/* ========================================================================= */

/* Ewald lattice sum of the Coulomb potential (Ewald 1921), splitting        */
/* parameter beta:                                                           */
/*   Psi(r) = sum_p erfc(beta |r + P p|)/|r + P p|                           */
/*          + (4 pi / V) sum_{k != 0} exp(-k^2 / (4 beta^2)) / k^2 cos(k.r)  */
/*          - pi / (V beta^2),                                               */
/* k = 2 pi (n_x/len_x, n_y/len_y, n_z/len_z); and at r = 0 its regular part */
/*   Psi_0 = lim_{r->0} (Psi(r) - 1/r)                                       */
/*         = sum_{p != 0} erfc(beta |P p|)/|P p| + (4 pi / V) sum_k ...      */
/*           - 2 beta / sqrt(pi) - pi / (V beta^2).                          */
/* Terms are dropped below 1e-16 of the leading ones: images within          */
/* 6.2 / beta, wave vectors with k^2 / (4 beta^2) <= 38.                     */
typedef struct {
  double len[3], V, beta, rc, kc2;
  int pmax[3], kmax[3];
} ewald_t;

static void ewald_init(ewald_t* E, const double len[3], double beta) {
  E->V = len[0] * len[1] * len[2];
  E->beta = beta;
  E->rc = 6.2 / beta;
  E->kc2 = 4.0 * beta * beta * 38.0;
  for (int d = 0; d < 3; ++d) {
    E->len[d] = len[d];
    E->pmax[d] = (int)ceil(E->rc / len[d]) + 1;
    E->kmax[d] = (int)ceil(sqrt(E->kc2) * len[d] / (2.0 * OR_PI));
  }
}

/* r: displacement; zero: r is a lattice point's own node (returns Psi_0) */
static double ewald_psi(const ewald_t* E, const double r[3], int zero) {
  double s = 0.0;
  for (int pz = -E->pmax[2]; pz <= E->pmax[2]; ++pz)
    for (int py = -E->pmax[1]; py <= E->pmax[1]; ++py)
      for (int px = -E->pmax[0]; px <= E->pmax[0]; ++px) {
        if (zero && px == 0 && py == 0 && pz == 0) continue;
        double dx = r[0] + px * E->len[0], dy = r[1] + py * E->len[1], dz = r[2] + pz * E->len[2];
        double rr = sqrt(dx * dx + dy * dy + dz * dz);
        if (rr < E->rc) s += erfc(E->beta * rr) / rr;
      }
  double sk = 0.0;
  for (int nz = -E->kmax[2]; nz <= E->kmax[2]; ++nz)
    for (int ny = -E->kmax[1]; ny <= E->kmax[1]; ++ny)
      for (int nx = -E->kmax[0]; nx <= E->kmax[0]; ++nx) {
        if (nx == 0 && ny == 0 && nz == 0) continue;
        double kx = 2.0 * OR_PI * nx / E->len[0], ky = 2.0 * OR_PI * ny / E->len[1];
        double kz = 2.0 * OR_PI * nz / E->len[2];
        double k2 = kx * kx + ky * ky + kz * kz;
        if (k2 > E->kc2) continue;
        sk += exp(-k2 / (4.0 * E->beta * E->beta)) / k2 * cos(kx * r[0] + ky * r[1] + kz * r[2]);
      }
  s += 4.0 * OR_PI / E->V * sk - OR_PI / (E->V * E->beta * E->beta);
  if (zero) s -= 2.0 * E->beta / sqrt(OR_PI);
  return s;
}

typedef struct {
  ctx_t C;                         /* a, h, order, m, levels, lo, len, ke and gamma */
  int n[OR_MAX_LEVELS][3];         /* nodes per level and dimension */
  size_t off[OR_MAX_LEVELS + 1];   /* first node of each level in the concatenated grids */
  double* K;                       /* top-level kernel, K[(dz n + dy) n + dx] for node offsets d */
} pctx_t;

static int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

static size_t pidx(const pctx_t* P, int k, int ix, int iy, int iz) {
  const int* n = P->n[k];
  return P->off[k] + ((size_t)wrapi(iz, n[2]) * n[1] + (size_t)wrapi(iy, n[1])) * n[0] + (size_t)wrapi(ix, n[0]);
}

/* nodes per dimension (len / h, an integer) and level count: as given (every */
/* level must halve), else the fewest levels whose top grid has at most 8     */
/* nodes per side, stopping where a level cannot halve                         */
static int periodic_shape(const oracle_params* p, int n0[3], int* levels) {
  if (!(p->a > 0.0) || !(p->h > 0.0) || !isfinite(p->a) || !isfinite(p->h)) return OR_EINVAL;
  for (int d = 0; d < 3; ++d) {
    if (!(p->len[d] > 0.0) || !isfinite(p->len[d])) return OR_EINVAL;
    double t = p->len[d] / p->h;
    long r = lround(t);
    if (r < 1 || fabs(t - (double)r) > 1e-9 * t || r > (1 << 20)) return OR_EINVAL;
    if (2.0 * p->a > p->len[d]) return OR_EINVAL;
    n0[d] = (int)r;
  }
  int l = p->levels;
  if (l == 0) {
    l = 1;
    for (;;) {
      int big = 0, even = 1;
      for (int d = 0; d < 3; ++d) {
        int nk = n0[d] >> (l - 1);
        if (nk > 8) big = 1;
        if (nk % 2) even = 0;
      }
      if (!big || !even || l == OR_MAX_LEVELS) break;
      ++l;
    }
  }
  if (l < 1 || l > OR_MAX_LEVELS) return OR_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (n0[d] % (1 << (l - 1))) return OR_EINVAL;
  *levels = l;
  return OR_OK;
}

int oracle_periodic_layout(const oracle_params* p, int* levels, int* gn /* [L][3] */) {
  int n0[3], l;
  int rc = periodic_shape(p, n0, &l);
  if (rc) return rc;
  *levels = l;
  for (int k = 0; k < l; ++k)
    for (int d = 0; d < 3; ++d) gn[3 * k + d] = n0[d] >> k;
  return OR_OK;
}

static int pctx_init(pctx_t* P, const oracle_params* p) {
  memset(P, 0, sizeof(*P));
  int n0[3], l;
  int rc = periodic_shape(p, n0, &l);
  if (rc) return rc;
  oracle_params q = *p;
  q.levels = l;
  rc = ctx_init(&P->C, &q);           /* scalars and gamma; its free-space ranges go unused */
  if (rc) return rc;
  P->off[0] = 0;
  for (int k = 0; k < l; ++k) {
    for (int d = 0; d < 3; ++d) P->n[k][d] = n0[d] >> k;
    P->off[k + 1] = P->off[k] + (size_t)P->n[k][0] * P->n[k][1] * P->n[k][2];
  }
  /* top-level kernel table */
  const int t = l - 1;
  const int* nt = P->n[t];
  const size_t nn = (size_t)nt[0] * nt[1] * nt[2];
  if (nn > 32768) return OR_EINVAL;
  P->K = (double*)malloc(sizeof(double) * nn);
  const double ht = ldexp(P->C.h, t), aL = ldexp(P->C.a, t);
  double lmin = P->C.len[0];
  for (int d = 1; d < 3; ++d) if (P->C.len[d] < lmin) lmin = P->C.len[d];
  ewald_t E;
  ewald_init(&E, P->C.len, 2.5 / lmin);
  int im[3];
  for (int d = 0; d < 3; ++d) im[d] = (int)ceil(aL / P->C.len[d]) + 1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < (int)nn; ++e) {
    int dx = e % nt[0], dy = (e / nt[0]) % nt[1], dz = e / (nt[0] * nt[1]);
    double r[3] = {ht * dx, ht * dy, ht * dz};
    int zero = (dx == 0 && dy == 0 && dz == 0);
    double s = ewald_psi(&E, r, zero);
    if (zero) s += g_level(&P->C, t, 0.0);
    for (int pz = -im[2]; pz <= im[2]; ++pz)
      for (int py = -im[1]; py <= im[1]; ++py)
        for (int px = -im[0]; px <= im[0]; ++px) {
          if (zero && px == 0 && py == 0 && pz == 0) continue;
          double vx = r[0] + px * P->C.len[0], vy = r[1] + py * P->C.len[1], vz = r[2] + pz * P->C.len[2];
          double rho = sqrt(vx * vx + vy * vy + vz * vz);
          if (rho < aL) s -= 1.0 / rho - g_level(&P->C, t, rho);
        }
    P->K[e] = s;
  }
  return OR_OK;
}

/* position mapped into [lo, lo + len) */
static double wrap_pos(double x, double lo, double len) { return x - len * floor((x - lo) / len); }

/* Periodic MSM: the stages above with node indices modulo n_k, the pair sum */
/* over images and the top level through K.  Same outputs and conventions as */
/* oracle_msm (grids: the periodic level grids, oracle_periodic_layout       */
/* order, x fastest); the virial is sum_i (r_i - lo) F_i with r_i mapped     */
/* into the box.                                                             */
int oracle_msm_periodic(const oracle_params* p, int n, const double* x, const double* y, const double* z,
                        const double* q, double* fx, double* fy, double* fz, double* phi, double* energy,
                        double* virial, double* qgrid, double* ucut, double* ugrid, double* phis_out,
                        int nthreads) {
  pctx_t P;
  int rc = pctx_init(&P, p);
  if (rc) { free(P.K); return rc; }
  const ctx_t* C = &P.C;
  if (n < 0 || (n > 0 && (!x || !y || !z || !q))) { free(P.K); return OR_EINVAL; }
  for (int i = 0; i < n; ++i)
    if (!isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i]) || !isfinite(q[i])) { free(P.K); return OR_ENONFINITE; }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  const int l = C->levels, no = C->order, half = C->order / 2, R = C->order - 1;
  size_t na = (size_t)(n > 0 ? n : 1);
  double* w3[3];
  for (int d = 0; d < 3; ++d) w3[d] = (double*)malloc(sizeof(double) * na);
  for (int i = 0; i < n; ++i) {
    w3[0][i] = wrap_pos(x[i], C->lo[0], C->len[0]);
    w3[1][i] = wrap_pos(y[i], C->lo[1], C->len[1]);
    w3[2][i] = wrap_pos(z[i], C->lo[2], C->len[2]);
  }
  size_t ng = P.off[l];
  double* qg = (double*)calloc(ng, sizeof(double));
  double* uc = (double*)calloc(ng, sizeof(double));
  double* ug = (double*)calloc(ng, sizeof(double));
  double* ps = (double*)calloc(na, sizeof(double));
  double* fs[3], *gl[3];
  for (int d = 0; d < 3; ++d) { fs[d] = (double*)calloc(na, sizeof(double)); gl[d] = (double*)calloc(na, sizeof(double)); }
  double* pl = (double*)calloc(na, sizeof(double));
  int bad = 0;

  /* short range: every pair at its nearest image, brute force */
  const double a2 = C->a * C->a;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
  for (int i = 0; i < n; ++i) {
    double s = 0.0, f[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double dv[3], r2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        dv[d] = w3[d][i] - w3[d][j];
        dv[d] -= C->len[d] * nearbyint(dv[d] / C->len[d]);
        r2 += dv[d] * dv[d];
      }
      if (r2 >= a2) continue;
      if (r2 == 0.0) { bad = 1; continue; }
      double rr = sqrt(r2);
      s += q[j] * g_short(C, rr);
      double w = -q[i] * q[j] * dg_short(C, rr) / rr;
      for (int d = 0; d < 3; ++d) f[d] += w * dv[d];
    }
    ps[i] = s;
    for (int d = 0; d < 3; ++d) fs[d][i] = f[d];
  }
  if (bad) { rc = OR_ECOINCIDENT; goto pdone; }

  /* anterpolation (serial, atom order) */
  for (int i = 0; i < n; ++i) {
    double t[3], w[3][8];
    int f[3];
    for (int d = 0; d < 3; ++d) {
      t[d] = (w3[d][i] - C->lo[d]) / C->h;
      f[d] = (int)floor(t[d]);
      for (int s = 0; s < no; ++s) w[d][s] = oracle_Phi(no, t[d] - (f[d] - (half - 1) + s));
    }
    for (int sz = 0; sz < no; ++sz)
      for (int sy = 0; sy < no; ++sy)
        for (int sx = 0; sx < no; ++sx)
          qg[pidx(&P, 0, f[0] - (half - 1) + sx, f[1] - (half - 1) + sy, f[2] - (half - 1) + sz)] +=
              q[i] * w[0][sx] * w[1][sy] * w[2][sz];
  }
  /* restriction */
  for (int k = 0; k + 1 < l; ++k) {
    const int* cn = P.n[k + 1];
#pragma omp parallel for collapse(2) schedule(static)
    for (int mz = 0; mz < cn[2]; ++mz)
      for (int my = 0; my < cn[1]; ++my)
        for (int mx = 0; mx < cn[0]; ++mx) {
          double s = 0.0;
          for (int vz = 2 * mz - R; vz <= 2 * mz + R; ++vz) {
            double wz = oracle_Phi(no, 0.5 * vz - mz);
            for (int vy = 2 * my - R; vy <= 2 * my + R; ++vy) {
              double wy = oracle_Phi(no, 0.5 * vy - my);
              for (int vx = 2 * mx - R; vx <= 2 * mx + R; ++vx) {
                double wx = oracle_Phi(no, 0.5 * vx - mx);
                s += wx * wy * wz * qg[pidx(&P, k, vx, vy, vz)];
              }
            }
          }
          qg[pidx(&P, k + 1, mx, my, mz)] = s;
        }
  }
  /* lattice cutoff below the top: every image of each node pair closer than 2^{k+1} a */
  const int H = (int)ceil(2.0 * C->a / C->h);
  for (int k = 0; k + 1 < l; ++k) {
    const int* nk = P.n[k];
    const double hk = ldexp(C->h, k), rcut = ldexp(C->a, k + 1);
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int mz = 0; mz < nk[2]; ++mz)
      for (int my = 0; my < nk[1]; ++my)
        for (int mx = 0; mx < nk[0]; ++mx) {
          double s = 0.0;
          for (int sz = -H; sz <= H; ++sz)
            for (int sy = -H; sy <= H; ++sy)
              for (int sx = -H; sx <= H; ++sx) {
                double d = hk * sqrt((double)(sx * sx + sy * sy + sz * sz));
                if (d >= rcut) continue;
                s += g_level(C, k, d) * qg[pidx(&P, k, mx + sx, my + sy, mz + sz)];
              }
          uc[pidx(&P, k, mx, my, mz)] = s;
        }
  }
  /* top level through the periodic kernel */
  {
    const int t = l - 1;
    const int* nt = P.n[t];
#pragma omp parallel for collapse(2) schedule(static)
    for (int mz = 0; mz < nt[2]; ++mz)
      for (int my = 0; my < nt[1]; ++my)
        for (int mx = 0; mx < nt[0]; ++mx) {
          double s = 0.0;
          for (int vz = 0; vz < nt[2]; ++vz)
            for (int vy = 0; vy < nt[1]; ++vy)
              for (int vx = 0; vx < nt[0]; ++vx)
                s += P.K[((size_t)wrapi(mz - vz, nt[2]) * nt[1] + wrapi(my - vy, nt[1])) * nt[0] +
                         wrapi(mx - vx, nt[0])] * qg[pidx(&P, t, vx, vy, vz)];
          uc[pidx(&P, t, mx, my, mz)] = s;
        }
  }
  memcpy(ug, uc, ng * sizeof(double));
  /* prolongation */
  for (int k = l - 2; k >= 0; --k) {
    const int* nk = P.n[k];
#pragma omp parallel for collapse(2) schedule(static)
    for (int mz = 0; mz < nk[2]; ++mz)
      for (int my = 0; my < nk[1]; ++my)
        for (int mx = 0; mx < nk[0]; ++mx) {
          double s = 0.0;
          for (int vz = (mz - R + 1) >> 1; 2 * vz <= mz + R; ++vz) {
            if (abs(mz - 2 * vz) > R) continue;
            double wz = oracle_Phi(no, 0.5 * mz - vz);
            for (int vy = (my - R + 1) >> 1; 2 * vy <= my + R; ++vy) {
              if (abs(my - 2 * vy) > R) continue;
              double wy = oracle_Phi(no, 0.5 * my - vy);
              for (int vx = (mx - R + 1) >> 1; 2 * vx <= mx + R; ++vx) {
                if (abs(mx - 2 * vx) > R) continue;
                double wx = oracle_Phi(no, 0.5 * mx - vx);
                s += wx * wy * wz * ug[pidx(&P, k + 1, vx, vy, vz)];
              }
            }
          }
          ug[pidx(&P, k, mx, my, mz)] += s;
        }
  }
  /* interpolation */
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    double t[3], w[3][8], dw[3][8];
    int f[3];
    for (int d = 0; d < 3; ++d) {
      t[d] = (w3[d][i] - C->lo[d]) / C->h;
      f[d] = (int)floor(t[d]);
      for (int e = 0; e < no; ++e) {
        double u = t[d] - (f[d] - (half - 1) + e);
        w[d][e] = oracle_Phi(no, u);
        dw[d][e] = oracle_dPhi(no, u) / C->h;
      }
    }
    double pv = 0.0, a0 = 0.0, a1 = 0.0, a2v = 0.0;
    for (int sz = 0; sz < no; ++sz)
      for (int sy = 0; sy < no; ++sy)
        for (int sx = 0; sx < no; ++sx) {
          double u = ug[pidx(&P, 0, f[0] - (half - 1) + sx, f[1] - (half - 1) + sy, f[2] - (half - 1) + sz)];
          pv += w[0][sx] * w[1][sy] * w[2][sz] * u;
          a0 += dw[0][sx] * w[1][sy] * w[2][sz] * u;
          a1 += w[0][sx] * dw[1][sy] * w[2][sz] * u;
          a2v += w[0][sx] * w[1][sy] * dw[2][sz] * u;
        }
    pl[i] = pv; gl[0][i] = a0; gl[1][i] = a1; gl[2][i] = a2v;
  }
  {
    const double self = gamma_eval(C->c, C->m, 0.0) / C->a;
    nsum_t e = {0.0, 0.0};
    nsum_t w[9];
    memset(w, 0, sizeof(w));
    for (int i = 0; i < n; ++i) {
      double ph = C->ke * (ps[i] + pl[i] - q[i] * self);
      double f3[3], r3[3];
      for (int d = 0; d < 3; ++d) {
        f3[d] = C->ke * (fs[d][i] - q[i] * gl[d][i]);
        r3[d] = w3[d][i] - C->lo[d];
      }
      if (phi) phi[i] = ph;
      if (fx) fx[i] = f3[0];
      if (fy) fy[i] = f3[1];
      if (fz) fz[i] = f3[2];
      if (phis_out) phis_out[i] = C->ke * ps[i];
      nsum_add(&e, 0.5 * q[i] * ph);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) nsum_add(&w[3 * a + b], r3[a] * f3[b]);
    }
    if (energy) *energy = e.s + e.c;
    if (virial)
      for (int t = 0; t < 9; ++t) virial[t] = w[t].s + w[t].c;
  }
  if (qgrid) memcpy(qgrid, qg, ng * sizeof(double));
  if (ucut) memcpy(ucut, uc, ng * sizeof(double));
  if (ugrid) memcpy(ugrid, ug, ng * sizeof(double));
pdone:
  free(P.K); free(qg); free(uc); free(ug); free(ps); free(pl);
  for (int d = 0; d < 3; ++d) { free(w3[d]); free(fs[d]); free(gl[d]); }
  return rc;
}

/* Periodic top-level kernel K at the node offsets of the top grid (the table */
/* oracle_msm_periodic uses), for the pins.                                   */
int oracle_periodic_top_kernel(const oracle_params* p, double* K, int cap) {
  pctx_t P;
  int rc = pctx_init(&P, p);
  if (!rc) {
    const int* nt = P.n[P.C.levels - 1];
    size_t nn = (size_t)nt[0] * nt[1] * nt[2];
    if ((size_t)cap < nn) rc = OR_EINVAL;
    else memcpy(K, P.K, nn * sizeof(double));
  }
  free(P.K);
  return rc;
}

/* Ewald summation of point charges in the periodic box (Ewald 1921): the    */
/* exact periodic Coulomb energy, potentials and forces the periodic method  */
/* approximates.  phi_i = sum_{(j,p) != (i,0)} q_j Psi-terms, E = 1/2 sum    */
/* q_i phi_i, F_i = -q_i grad phi_i.  beta = 12 / min(len), so the real-space */
/* part needs only each pair's nearest image (6.2 / beta < min(len) / 2).     */
int oracle_ewald(int n, const double* x, const double* y, const double* z, const double* q,
                 const double* lo, const double* len, double ke, double* fx, double* fy, double* fz,
                 double* phi, double* energy, int nthreads) {
  if (n < 0 || (n > 0 && (!x || !y || !z || !q)) || !lo || !len) return OR_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (!(len[d] > 0.0) || !isfinite(len[d]) || !isfinite(lo[d])) return OR_EINVAL;
  if (ke == 0.0) ke = 1.0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  double lmin = len[0];
  for (int d = 1; d < 3; ++d) if (len[d] < lmin) lmin = len[d];
  ewald_t E;
  ewald_init(&E, len, 12.4 / lmin);
  const double beta = E.beta, V = E.V;
  size_t na = (size_t)(n > 0 ? n : 1);
  double* r[3];
  for (int d = 0; d < 3; ++d) r[d] = (double*)malloc(sizeof(double) * na);
  for (int i = 0; i < n; ++i) {
    r[0][i] = wrap_pos(x[i], lo[0], len[0]);
    r[1][i] = wrap_pos(y[i], lo[1], len[1]);
    r[2][i] = wrap_pos(z[i], lo[2], len[2]);
  }
  /* wave vectors and structure factors S(k) = sum_j q_j exp(i k.r_j) */
  int nk = 0, cap = (2 * E.kmax[0] + 1) * (2 * E.kmax[1] + 1) * (2 * E.kmax[2] + 1);
  double* kv = (double*)malloc(sizeof(double) * 4 * (size_t)cap);
  for (int nz = -E.kmax[2]; nz <= E.kmax[2]; ++nz)
    for (int ny = -E.kmax[1]; ny <= E.kmax[1]; ++ny)
      for (int nx = -E.kmax[0]; nx <= E.kmax[0]; ++nx) {
        if (nx == 0 && ny == 0 && nz == 0) continue;
        double kx = 2.0 * OR_PI * nx / len[0], ky = 2.0 * OR_PI * ny / len[1], kz = 2.0 * OR_PI * nz / len[2];
        double k2 = kx * kx + ky * ky + kz * kz;
        if (k2 > E.kc2) continue;
        kv[4 * nk] = kx; kv[4 * nk + 1] = ky; kv[4 * nk + 2] = kz;
        kv[4 * nk + 3] = exp(-k2 / (4.0 * beta * beta)) / k2;
        ++nk;
      }
  double* sre = (double*)calloc((size_t)(nk > 0 ? nk : 1), sizeof(double));
  double* sim = (double*)calloc((size_t)(nk > 0 ? nk : 1), sizeof(double));
#pragma omp parallel for schedule(static)
  for (int t = 0; t < nk; ++t) {
    double a = 0.0, b = 0.0;
    for (int j = 0; j < n; ++j) {
      double ph = kv[4 * t] * r[0][j] + kv[4 * t + 1] * r[1][j] + kv[4 * t + 2] * r[2][j];
      a += q[j] * cos(ph);
      b += q[j] * sin(ph);
    }
    sre[t] = a; sim[t] = b;
  }
  double Q = 0.0;
  for (int j = 0; j < n; ++j) Q += q[j];
  double* ph_ = (double*)malloc(sizeof(double) * na);
  double* f_ = (double*)malloc(sizeof(double) * 3 * na);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
  for (int i = 0; i < n; ++i) {
    double p = 0.0, f[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double dv[3], r2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        dv[d] = r[d][i] - r[d][j];
        dv[d] -= len[d] * nearbyint(dv[d] / len[d]);
        r2 += dv[d] * dv[d];
      }
      if (r2 == 0.0) { bad = 1; continue; }
      double rr = sqrt(r2);
      if (rr >= E.rc) continue;
      double ec = erfc(beta * rr);
      p += q[j] * ec / rr;
      double w = q[j] * (ec / rr + 2.0 * beta / sqrt(OR_PI) * exp(-beta * beta * r2)) / r2;
      for (int d = 0; d < 3; ++d) f[d] += w * dv[d];
    }
    double pk = 0.0, g[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < nk; ++t) {
      double th = kv[4 * t] * r[0][i] + kv[4 * t + 1] * r[1][i] + kv[4 * t + 2] * r[2][i];
      double c = cos(th), s = sin(th);
      /* Re(exp(-i th) S) = c Sre + s Sim;  Im(exp(-i th) S) = c Sim - s Sre */
      double re = c * sre[t] + s * sim[t], im = c * sim[t] - s * sre[t];
      pk += kv[4 * t + 3] * re;
      for (int d = 0; d < 3; ++d) g[d] += kv[4 * t + 3] * kv[4 * t + d] * im;
    }
    p += 4.0 * OR_PI / V * pk - 2.0 * beta / sqrt(OR_PI) * q[i] - OR_PI * Q / (V * beta * beta);
    ph_[i] = ke * p;
    for (int d = 0; d < 3; ++d) f_[3 * (size_t)i + d] = ke * q[i] * (f[d] - 4.0 * OR_PI / V * g[d]);
  }
  nsum_t e = {0.0, 0.0};
  for (int i = 0; i < n; ++i) {
    nsum_add(&e, 0.5 * q[i] * ph_[i]);
    if (phi) phi[i] = ph_[i];
    if (fx) fx[i] = f_[3 * (size_t)i];
    if (fy) fy[i] = f_[3 * (size_t)i + 1];
    if (fz) fz[i] = f_[3 * (size_t)i + 2];
  }
  if (energy) *energy = e.s + e.c;
  for (int d = 0; d < 3; ++d) free(r[d]);
  free(kv); free(sre); free(sim); free(ph_); free(f_);
  return bad ? OR_ECOINCIDENT : OR_OK;
}
