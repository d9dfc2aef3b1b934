// Host side of libmsm: parameter validation, grid hierarchy, stencil and
// top-level tables (double precision on the host), workspace layout, and the
// C ABI declared in include/msm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <utility>
#include <cmath>
#include <cstring>
#include <new>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "msm_plan.hpp"

namespace {
thread_local std::string g_last_error;
}  // namespace

msm_status fail(msm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

msm_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return MSM_ERR_HIP;
}

// Create (once per owner) the auxiliary stream and fork/join events on the
// current device.  Streams keep the default priority.
hipError_t ensure_aux(AuxStreams& A) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (A.cc.shortr.stream && A.device == dev) return hipSuccess;
  destroy_aux(A);
  // the events only order work between streams of this device: no timing and
  // no system-scope fence (kernels end with a device-scope release already)
  const unsigned ev_flags = hipEventDisableTiming | hipEventDisableSystemFence;
  for (msm::SideStream* ss : {&A.cc.shortr, &A.cc.lattice0}) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ss->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ss->fork, ev_flags);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ss->join, ev_flags);
  }
  if (e != hipSuccess) {
    destroy_aux(A);
    return e;
  }
  A.device = dev;
  return hipSuccess;
}

void destroy_aux(AuxStreams& A) {
  for (msm::SideStream* ss : {&A.cc.shortr, &A.cc.lattice0}) {
    if (ss->stream) (void)hipStreamDestroy(ss->stream);
    if (ss->fork) (void)hipEventDestroy(ss->fork);
    if (ss->join) (void)hipEventDestroy(ss->join);
  }
  A = AuxStreams{};
}

namespace {

// Taylor smoothing (Sec. 2.3): gamma(rho) = sum_k c_k rho^{2k}, rho < 1, with c_k
// the coefficients of the degree-m Taylor polynomial of s^{-1/2} at s = 1,
// collected in powers of s.
void taylor_coeffs(int m, double* c) {
  for (int k = 0; k <= m; ++k) c[k] = 0.0;
  double tj = 1.0;                                   // binom(-1/2, j)
  for (int j = 0; j <= m; ++j) {
    if (j > 0) tj *= (-0.5 - (j - 1)) / j;
    double bjk = 1.0;                                // binom(j, k)
    for (int k = 0; k <= j; ++k) {
      if (k > 0) bjk = bjk * (j - k + 1) / k;
      c[k] += tj * bjk * (((j - k) % 2) ? -1.0 : 1.0);
    }
  }
}

double gamma_h(const double* c, int m, double rho) {
  if (rho >= 1.0) return 1.0 / rho;
  double s = rho * rho, v = c[m];
  for (int k = m - 1; k >= 0; --k) v = v * s + c[k];
  return v;
}


int floor_div2(int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); }
int ceil_div2(int v) { return -floor_div2(-v); }

// Top level of a periodic plan: K(d) = sum over images p of g^{l-1}(|h_t d + P p|)
// for every node offset d of the top grid (P = diag(box edges)).  g^{l-1}
// decays as 1/r, so the image sum is the Ewald one (conducting boundary,
// uniform neutralising background): K = Psi - sum over the images closer than
// A = 2^{l-1} a of (1/rho - g^{l-1}(rho)), with
//   Psi(r) = sum_p erfc(b |r + P p|) / |r + P p|
//          + (4 pi / V) sum_{k != 0} exp(-k^2 / 4b^2) cos(k.r) / k^2 - pi / (V b^2)
// and, at d = 0, the node's own term g^{l-1}(0) in place of the singular
// p = 0 Coulomb term (whose Ewald remainder is -2b/sqrt(pi)).  b = 3 / min(len);
// real-space images to 6 / b and wave vectors to k^2 = 156 b^2 leave terms
// below 1e-16.
void periodic_top_table(const double* c, int m, double A, double ht, const int nt[3], const double len[3],
                        std::vector<double>& K) {
  const double pi = 3.14159265358979323846;
  const double lmin = std::min({len[0], len[1], len[2]});
  const double b = 3.0 / lmin, V = len[0] * len[1] * len[2], rc = 6.0 / b, kc2 = 156.0 * b * b;
  struct Wave { double kx, ky, kz, w; };
  std::vector<Wave> waves;
  int kn[3], pn[3], an[3];
  for (int d = 0; d < 3; ++d) {
    kn[d] = (int)std::ceil(std::sqrt(kc2) * len[d] / (2.0 * pi));
    pn[d] = (int)std::ceil(rc / len[d]) + 1;
    an[d] = (int)std::ceil(A / len[d]) + 1;
  }
  for (int iz = -kn[2]; iz <= kn[2]; ++iz)
    for (int iy = -kn[1]; iy <= kn[1]; ++iy)
      for (int ix = -kn[0]; ix <= kn[0]; ++ix) {
        if (!ix && !iy && !iz) continue;
        const Wave v{2.0 * pi * ix / len[0], 2.0 * pi * iy / len[1], 2.0 * pi * iz / len[2], 0.0};
        const double k2 = v.kx * v.kx + v.ky * v.ky + v.kz * v.kz;
        if (k2 <= kc2) waves.push_back(Wave{v.kx, v.ky, v.kz, 4.0 * pi / V * std::exp(-k2 / (4.0 * b * b)) / k2});
      }
  K.assign((size_t)nt[0] * nt[1] * nt[2], 0.0);
  for (int dz = 0; dz < nt[2]; ++dz)
    for (int dy = 0; dy < nt[1]; ++dy)
      for (int dx = 0; dx < nt[0]; ++dx) {
        const double r[3] = {ht * dx, ht * dy, ht * dz};
        const bool self = !dx && !dy && !dz;
        double real = 0.0, corr = 0.0, recip = 0.0;
        // images within the Ewald real-space cutoff and within A, one pass each
        for (int pz = -std::max(pn[2], an[2]); pz <= std::max(pn[2], an[2]); ++pz)
          for (int py = -std::max(pn[1], an[1]); py <= std::max(pn[1], an[1]); ++py)
            for (int px = -std::max(pn[0], an[0]); px <= std::max(pn[0], an[0]); ++px) {
              if (self && !px && !py && !pz) continue;
              const double vx = r[0] + px * len[0], vy = r[1] + py * len[1], vz = r[2] + pz * len[2];
              const double rho = std::sqrt(vx * vx + vy * vy + vz * vz);
              if (rho < rc) real += std::erfc(b * rho) / rho;
              if (rho < A) corr += 1.0 / rho - gamma_h(c, m, rho / A) / A;
            }
        for (const Wave& v : waves) recip += v.w * std::cos(v.kx * r[0] + v.ky * r[1] + v.kz * r[2]);
        double k = real + recip - pi / (V * b * b) - corr;
        if (self) k += gamma_h(c, m, 0.0) / A - 2.0 * b / std::sqrt(pi);
        K[((size_t)dz * nt[1] + dy) * nt[0] + dx] = k;
      }
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Largest number of lanes of one half-wave (32 lanes) whose window offsets
// fall in the same LDS bank (32 banks of 4 bytes).
int bank_conflicts(int xl, int ty, int tz, int B, int px, int pp) {
  int worst = 0;
  for (int half = 0; half < 2; ++half) {
    int cnt[32] = {0};
    for (int l = half * 32; l < half * 32 + 32; ++l) {
      const int xi = l % xl, yi = (l / xl) % ty, zi = l / (xl * ty);
      if (zi >= tz) continue;
      const int off = zi * pp + yi * px + xi * B;
      worst = std::max(worst, ++cnt[off & 31]);
    }
  }
  return worst;
}

// Row and plane pitches (floats) of a window tile of `planes` z planes with
// the fewest bank conflicts whose window still fits in max_floats.
void pad_window(msm::LatTile& t, int B, int H, int planes, int max_floats) {
  const int WX = t.xl * B + 2 * H, PY = t.ty + 2 * H;
  int best = 1 << 30;
  t.px = WX;
  t.pp = PY * WX;
  for (int px = WX; px < WX + 32; ++px)
    for (int extra = 0; extra < 32; ++extra) {
      const int pp = PY * px + extra;
      if (planes * pp > max_floats) continue;
      const int c = bank_conflicts(t.xl, t.ty, t.tz, B, px, pp);
      const int score = c * 4096 + (pp * planes - WX * PY * planes) / 64;
      if (score < best) {
        best = score;
        t.px = px;
        t.pp = pp;
      }
    }
}

// Split the compact rows (sorted by nz) into G contiguous nz ranges of nearly
// equal work; grp[g] = first row of group g, grp[G] = number of rows.  Returns
// the largest nz span (nz_hi - nz_lo) of a group.
int split_rows(const std::vector<int4>& rows, int B, int G, short* grp) {
  const int n = (int)rows.size();
  std::vector<double> cost(n);
  double total = 0.0;
  for (int r = 0; r < n; ++r) {
    const int xr = rows[r].z;
    cost[r] = (2.0 * xr + 1.0) * B + (rows[r].y ? B + 2.0 * xr : 0.0) + 8.0;
    total += cost[r];
  }
  int g = 0, span = 0, first = 0;
  double acc = 0.0;
  grp[0] = 0;
  for (int r = 0; r < n; ++r) {
    acc += cost[r];
    const bool nz_ends = (r + 1 == n) || rows[r + 1].x != rows[r].x;
    if (nz_ends && g + 1 < G && acc >= total * (g + 1) / G) {
      grp[++g] = (short)(r + 1);
      span = std::max(span, rows[r].x - rows[first].x);
      first = r + 1;
    }
  }
  span = std::max(span, rows[n - 1].x - rows[first].x);
  while (g + 1 < G) grp[++g] = (short)n;        // fewer nz values than groups: empty groups
  grp[G] = (short)n;
  return span;
}

// Tile shapes and row groups of the windowed lattice-cutoff kernel.  For each
// candidate B (outputs per lane along x) and each sub-top level, pick
// (xl, ty, tz) lanes minimising a per-tile cost in wave instructions (FMA
// slots including ragged-tile waste, about half a FMA per tap with mirror-row
// pairing, plus the window load).  Then split the rows of each tile into
// groups so that the blocks of a launch (level 0 alone; levels 1 .. l-2
// together) cover the 256 compute units with short blocks: the launch is
// estimated as ceil(blocks / 256) times its longest block.
void choose_lattice_tiles(const Geom& g, const std::vector<int4>& rows, int taps, int H_,
                          int tables_bytes, msm::LatLaunch& lat, int force_b = 0, int force_waves = 0) {
  const int n_rows = lat.n_rows, n_wc = lat.n_wc;
  std::memset(&lat, 0, sizeof(lat));
  lat.H = H_;
  lat.n_rows = n_rows;
  lat.n_wc = n_wc;
  if (g.levels < 2 || H_ > msm::kLatMaxHalo) return;
  const int max_floats = (msm::kLatMaxLds - tables_bytes) / 4;
  // periodic levels get their ghost copies from u^{k,cut} itself: no row groups
  const int gmax = g.periodic ? 1 : std::min(msm::kLatMaxGroups, 2 * H_ + 1);
  double best = 1e300;
  msm::LatLaunch cand;
  const int Bs[3] = {4, 6, 8};
  for (int bi = 0; bi < 3; ++bi) {
    const int B = Bs[bi];
    if (force_b && B != force_b) continue;
    cand = lat;
    cand.b = B;
    cand.n = g.levels - 1;
    int span[msm::kLatMaxGroups + 1] = {};
    for (int G = 1; G <= gmax; ++G) span[G] = split_rows(rows, B, G, cand.grp[G]);
    // per level: best tile by per-tile cost (all groups)
    double tile_cost[msm::kMaxLevels] = {};
    long long tiles[msm::kMaxLevels] = {};
    bool ok = true;
    for (int k = 0; k < g.levels - 1; ++k) {
      const msm::Level& L = g.lv[k];
      double lbest = 1e300;
      msm::LatTile tb{};
      for (int tz = 1; tz <= 16; ++tz)
        for (int ty = 1; ty <= 16; ++ty)
          for (int xl = 1; xl <= 16; ++xl) {
            if (xl * ty * tz > 64 || xl * ty * tz < 32) continue;
            const int WX = xl * B + 2 * H_, PY = ty + 2 * H_, WZ = tz + 2 * H_;
            if (WZ * PY * WX > max_floats) continue;
            const long long nt = (long long)((L.n[0] + xl * B - 1) / (xl * B)) *
                                 ((L.n[1] + ty - 1) / ty) * ((L.n[2] + tz - 1) / tz);
            const double c = (double)nt * (0.55 * B * taps + (double)WZ * PY * WX / 16.0);
            if (c < lbest) {
              lbest = c;
              tb = msm::LatTile{k, xl, ty, tz, (L.n[0] + xl * B - 1) / (xl * B), (L.n[1] + ty - 1) / ty,
                                (L.n[2] + tz - 1) / tz, 0, WX, WX * PY, 1, 0};
            }
          }
      if (lbest >= 1e300) {
        ok = false;
        break;
      }
      cand.t[k] = tb;
      tiles[k] = (long long)tb.ntx * tb.nty * tb.ntz;
      tile_cost[k] = lbest / (double)tiles[k];
    }
    if (!ok) continue;
    // cost of one block of level k with G groups
    auto block_cost = [&](int k, int G) {
      const msm::LatTile& t = cand.t[k];
      const int WX = t.xl * B + 2 * H_, PY = t.ty + 2 * H_;
      const double stage = (double)(t.tz + span[G]) * PY * WX / 16.0;
      return 0.55 * B * taps / G + stage + 300.0;
    };
    // groups per level for one launch over levels [k0, k1): a common target
    // block cost tau sets G_k = ceil(cost_k(1) / tau)
    auto choose_groups = [&](int k0, int k1) {
      double est_best = 1e300;
      int gbest[msm::kMaxLevels] = {};
      for (int kk = k0; kk < k1; ++kk)
        for (int G = 1; G <= gmax; ++G) {
          const double tau = block_cost(kk, G);
          int gk[msm::kMaxLevels] = {};
          long long blocks = 0;
          double longest = 0.0;
          for (int k = k0; k < k1; ++k) {
            int Gk = 1;
            while (Gk < gmax && block_cost(k, Gk) > tau) ++Gk;
            gk[k] = Gk;
            blocks += tiles[k] * Gk;
            longest = std::max(longest, block_cost(k, Gk));
          }
          const double est = (double)((blocks + 255) / 256) * longest;
          if (est < est_best) {
            est_best = est;
            std::copy(gk, gk + msm::kMaxLevels, gbest);
          }
        }
      for (int k = k0; k < k1; ++k) cand.t[k].groups = gbest[k];
      return est_best;
    };
    const double est = choose_groups(0, 1) + (g.levels > 2 ? choose_groups(1, g.levels - 1) : 0.0);
    // waves per block: a grid of many tiles balances its stencil rows better
    // over fewer waves per tile; a grid of few tiles needs every tile's waves
    cand.waves = force_waves ? force_waves
                             : (tiles[0] >= msm::kLatWavesTiles ? msm::kLatWavesFew : msm::kLatWavesMany);
    // padding, LDS, block and partial offsets
    long long blocks = 0;
    int lds_max = 0, part = 0;
    for (int k = 0; k < g.levels - 1; ++k) {
      msm::LatTile& t = cand.t[k];
      const int planes = t.tz + span[t.groups];
      pad_window(t, B, H_, planes, max_floats);
      const int lds = std::max(tables_bytes + planes * t.pp * 4, cand.waves * 64 * B * 8);
      lds_max = std::max(lds_max, lds);
      t.block0 = (int)blocks;
      blocks += tiles[k] * t.groups;
      t.part0 = part;
      if (t.groups > 1) part += t.groups * g.lv[k].count;
    }
    cand.lds_bytes = lds_max;
    cand.n_part = part;
    if (est < best) {
      best = est;
      lat = cand;
    }
  }
}

// Least squares min |A c - b| over the columns of A (rows x cols, row-major)
// by Householder reflections; A and b are overwritten.
void householder_lsq(std::vector<double>& A, std::vector<double>& b, int rows, int cols, double* c) {
  for (int k = 0; k < cols; ++k) {
    double norm = 0.0;
    for (int i = k; i < rows; ++i) norm += A[i * cols + k] * A[i * cols + k];
    norm = std::sqrt(norm);
    const double alpha = A[k * cols + k] > 0 ? -norm : norm;
    std::vector<double> v(rows - k);
    for (int i = k; i < rows; ++i) v[i - k] = A[i * cols + k];
    v[0] -= alpha;
    double vv = 0.0;
    for (double e : v) vv += e * e;
    if (vv == 0.0) continue;
    for (int j = k; j < cols; ++j) {
      double s = 0.0;
      for (int i = k; i < rows; ++i) s += v[i - k] * A[i * cols + j];
      s *= 2.0 / vv;
      for (int i = k; i < rows; ++i) A[i * cols + j] -= s * v[i - k];
    }
    double s = 0.0;
    for (int i = k; i < rows; ++i) s += v[i - k] * b[i];
    s *= 2.0 / vv;
    for (int i = k; i < rows; ++i) b[i] -= s * v[i - k];
  }
  for (int k = cols - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < cols; ++j) s -= A[k * cols + j] * c[j];
    c[k] = A[k * cols + k] != 0.0 ? s / A[k * cols + k] : 0.0;
  }
}

// The Wolf pair function's erfc on the device: erfc(x) = exp(-x^2) R(x), with
// the smooth scaled function R(x) = erfc(x) exp(x^2) written as a polynomial
// in t = 1 / (1 + x/2) (the substitution of Hastings' approximations in
// Abramowitz and Stegun 7.1.25-28), fitted here in double over x in [0, x_hi]
// by least squares in relative error.  The coefficients are rounded to float
// one at a time from t^0 up, the later ones refitted after each rounding, so
// the rounded polynomial keeps the fit's accuracy (about 1e-9 relative for
// x_hi <= 6) instead of carrying a fixed float-rounding bias into every pair.
// Returns the fitted polynomial's largest relative error on a fine grid.
double fit_wolf_erfc(double x_hi, float* ec) {
  constexpr int m = msm::kWolfTerms, n = 12 * msm::kWolfTerms;
  const double tmin = 1.0 / (1.0 + 0.5 * x_hi);
  std::vector<double> t(n), w(n);
  for (int i = 0; i < n; ++i) {
    const double z = std::cos(M_PI * (i + 0.5) / n);
    t[i] = tmin + 0.5 * (z + 1.0) * (1.0 - tmin);
    const double x = 2.0 * (1.0 / t[i] - 1.0);
    w[i] = 1.0 / (std::erfc(x) * std::exp(x * x));
  }
  double fixed[m];
  for (int k = 0; k < m; ++k) {
    const int cols = m - k;
    std::vector<double> A(n * cols), b(n);
    for (int i = 0; i < n; ++i) {
      double tp = 1.0, rhs = 1.0;
      for (int j = 0; j < m; ++j, tp *= t[i]) {
        if (j < k) rhs -= fixed[j] * tp * w[i];
        else A[i * cols + (j - k)] = tp * w[i];
      }
      b[i] = rhs;
    }
    double c[m];
    householder_lsq(A, b, n, cols, c);
    fixed[k] = (double)(float)c[0];
  }
  double worst = 0.0;
  for (int i = 0; i <= 4000; ++i) {
    const double x = x_hi * i / 4000.0, tt = 1.0 / (1.0 + 0.5 * x);
    double p = 0.0;
    for (int k = m - 1; k >= 0; --k) p = p * tt + fixed[k];
    worst = std::max(worst, std::fabs(p / (std::erfc(x) * std::exp(x * x)) - 1.0));
  }
  for (int k = 0; k < m; ++k) ec[k] = (float)fixed[k];
  return worst;
}

}  // namespace

void refresh_launch(msm_plan* P) {
  const Geom& g = P->g;
  msm::DevPtrs keep = P->desc.d;
  std::memset(&P->desc, 0, sizeof(P->desc));
  P->desc.d = keep;
  P->desc.g = g;
  P->desc.lat = P->lat;
  P->desc.atom_off = 0;
  P->desc.index = 0;
  P->desc.n_partials = P->n_partials;
  P->desc.n_rows = (int)P->rows.size();
  const msm::SysBlocks sb = msm::system_blocks(g, P->lat, P->n_partials);
  msm::LaunchGeom& lg = P->lg;
  lg = msm::LaunchGeom{};
  lg.n_sys = 1;
  lg.order = g.order;
  lg.m = g.m;
  lg.pair = g.pair;
  lg.lat_b = P->lat.b;
  lg.lat_waves = P->lat.b ? P->lat.waves : msm::kLatWavesMany;
  lg.lat_lds = P->lat.lds_bytes;
  lg.max_levels = g.levels;
  lg.streams = P->streams;
  lg.short_after = P->short_after;
  lg.short_split = P->short_split;
  lg.zero.blocks = sb.zero;
  lg.atoms.blocks = sb.atoms;
  lg.bin.blocks = sb.bin;
  lg.binrow.blocks = sb.binrow;
  lg.binrow_lds = msm::bin_rows_lds(g);
  lg.bin4 = g.bin_blocks == 0 && g.bin_row_blocks == 0 && g.binr_blocks == 0;
  lg.rchunk.blocks = sb.rchunk;
  lg.rscan.blocks = sb.rscan;
  lg.rsort.blocks = sb.rsort;
  lg.rsort_lds = msm::binr_sort_lds(g);
  lg.one.blocks = 1;
  lg.scan.blocks = sb.scan;
  lg.agather.blocks = sb.agather;
  lg.anterp_lds = msm::anterp_lds(g);
  // large grids: one prolongation launch per level instead of every block
  // rebuilding the coarser levels it reads (a level-0 tile of 8^3 nodes would
  // rebuild boxes of up to (2R + 3)^3 nodes on every coarser level)
  int tiles0 = 0;
  for (int k = 0; k + 1 < g.levels; ++k) {
    lg.prolong_level[k] = msm::prolong_level_blocks(g, k);
    if (k == 0) tiles0 = lg.prolong_level[k];
  }
  lg.prolong_split = g.levels > 1 && (tiles0 >= msm::kProlongSplitTiles || g.periodic);
  lg.periodic = g.periodic && !g.pair;
  lg.short_periodic = g.periodic != 0;
  for (int k = 0; k < g.levels; ++k) lg.ghost_blocks[k] = lg.periodic ? (g.lv[k].count + 255) / 256 : 0;
  lg.shortr.blocks = sb.shortr;
  lg.anterp.blocks = sb.anterp;
  lg.lattice0.blocks = sb.lattice0;
  lg.lattice.blocks = sb.lattice;
  lg.lattice_all.blocks = sb.lattice_all;
  lg.top.blocks = sb.top;
  lg.energy.blocks = sb.energy;
  for (int k = 0; k + 1 < g.levels; ++k) {
    lg.restrict_[k].blocks = sb.restrict_[k];
  }
  lg.prolong.blocks = sb.prolong;
}

// Neighbour cell rows (offsets oy, oz in [-reach, reach], row index
// (oz + reach) (2 reach + 1) + oy + reach) dealt to the 4 waves of a
// short-range block, largest expected x window first, each to the wave with
// the least work so far.  A row's expected window is the mean over atom
// positions (y, z) in a cell of 2 sqrt(a^2 - d^2), d the distance to the row.
// Free-space plans deal each row with its mirror (-oy, -oz) as one unit that
// a wave walks together: an atom near one face of its cell has a long window
// in the row beyond that face and a short one in the mirror row, so the sum
// of the two varies far less over the 64 atoms of a chunk than either.
void assign_short_rows(Geom& g) {
  const int R = g.reach, side = 2 * R + 1, nrows = side * side;
  const double a = g.a_win, cy = g.cs[1], cz = g.cs[2];
  std::vector<double> row_cost(nrows);
  for (int r = 0; r < nrows; ++r) {
    const int oy = r % side - R, oz = r / side - R;
    double sum = 0.0;
    const int K = 16;
    for (int iy = 0; iy < K; ++iy)
      for (int iz = 0; iz < K; ++iz) {
        const double y = (iy + 0.5) / K * cy, z = (iz + 0.5) / K * cz;
        auto gap = [](double v, int o, double c) {
          if (o > 0) return o * c - v;
          if (o < 0) return v - (o + 1) * c;
          return 0.0;
        };
        const double dy = gap(y, oy, cy), dz = gap(z, oz, cz), d2 = dy * dy + dz * dz;
        if (d2 < a * a) sum += 2.0 * std::sqrt(a * a - d2);
      }
    row_cost[r] = sum / (K * K) + 1.0;
  }
  // units: (cost, first row, second row or -1); the mirror of row r is nrows - 1 - r
  const bool pairs = !g.periodic;
  std::vector<std::tuple<double, int, int>> units;
  for (int r = 0; r < nrows; ++r) {
    const int m = nrows - 1 - r;
    if (pairs && m < r) continue;
    if (pairs && m > r) units.emplace_back(row_cost[r] + row_cost[m], r, m);
    else units.emplace_back(row_cost[r], r, -1);
  }
  std::sort(units.begin(), units.end(), [](const auto& x, const auto& y) {
    return std::get<0>(x) > std::get<0>(y) || (std::get<0>(x) == std::get<0>(y) && std::get<1>(x) < std::get<1>(y));
  });
  double load[msm::kShortWaves] = {};
  int count[msm::kShortWaves] = {};
  std::memset(g.short_rows, 0xff, sizeof(g.short_rows));
  std::memset(g.short_pair, 0xff, sizeof(g.short_pair));
  // a row r = (oz + R) side + oy + R is stored as its two offsets (R <= 4)
  auto code = [&](int r) { return (unsigned char)((r % side) | ((r / side) << 4)); };
  for (const auto& u : units) {
    int w = 0;
    for (int v = 1; v < msm::kShortWaves; ++v)
      if (count[v] < msm::kShortRowsPerWave && (count[w] >= msm::kShortRowsPerWave || load[v] < load[w])) w = v;
    g.short_rows[w][count[w]] = code(std::get<1>(u));
    if (std::get<2>(u) >= 0) g.short_pair[w][count[w]] = code(std::get<2>(u));
    ++count[w];
    load[w] += std::get<0>(u);
  }
}

// Short-range work items: each cell row's atoms are cut into 64-atom chunks;
// a row has row_items work items, item k taking chunks k, k + row_items, ...
// (sized for the row's expected atom count, so each item gets about
// item_chunks chunks; longer rows are still covered).
void set_row_items(Geom& g, int item_chunks) {
  g.item_chunks = std::max(1, item_chunks);
  const double per_row = (double)g.n_atoms / ((double)g.nc[1] * g.nc[2]);
  const int chunks = std::max(1, (int)std::ceil(per_row / 64.0));
  g.row_items = std::max(1, (chunks + g.item_chunks - 1) / g.item_chunks);
}

void set_short_blocks(Geom& g, int cap) {
  const int items = g.row_items * g.nc[1] * g.nc[2];
  g.short_blocks = cap > 0 ? std::min(cap, items) : items;
}

// Link cells of edge >= a / reach along y and z (kXSub times finer along x;
// coarser if the cell count would exceed 8 n + 4096), the short-range row
// assignment and work items, and the binning path the cells allow: one kernel
// for small systems whose blocks own few enough cells (unless the plan prefers
// the two-kernel path, as in batches), else two kernels when the cell counts of
// every block fit (LDS, histogram size), else four by cell row when the rows
// fit, else four over the cells.
void set_cell_geometry(msm_plan* P, int reach) {
  Geom& g = P->g;
  const msm_params& p = P->p;
  const int n_atoms = g.n_atoms;
  const double amargin = p.cutoff * (1.0 + 1e-4);
  auto set_cells = [&](int r, double edge_min) {
    g.reach = r;
    long long tot = 1;
    for (int d = 0; d < 3; ++d) {
      int nc = (int)std::floor(p.box_len[d] / (d == 0 ? edge_min / msm::kXSub : edge_min));
      nc = std::max(1, std::min(nc, d == 0 ? 4096 : 1024));
      g.nc[d] = nc;
      g.inv_cs[d] = (float)(nc / p.box_len[d]);
      g.cs[d] = (float)(p.box_len[d] / nc);
      tot *= nc;
    }
    return tot;
  };
  const long long cap = 8LL * std::max(n_atoms, 1) + 4096;
  long long nct = set_cells(reach, amargin / reach);
  for (int r = reach - 1; r >= 1 && nct > cap; --r) nct = set_cells(r, amargin / r);
  if (nct > cap) {
    const double vol = p.box_len[0] * p.box_len[1] * p.box_len[2];
    nct = set_cells(1, std::max(amargin, std::cbrt(vol / (double)cap)));
  }
  g.n_cells = (int)nct;
  assign_short_rows(g);
  const int rows = g.nc[1] * g.nc[2];
  const int nbr = std::min(rows, msm::kBinRowMaxBlocks);
  const long long own = (long long)((rows + nbr - 1) / nbr) * g.nc[0];
  const long long nb = (n_atoms + msm::kBinChunk - 1) / msm::kBinChunk;
  P->bin2_blocks = (n_atoms > 0 && g.n_cells <= msm::kBinMaxCells && nb * g.n_cells <= msm::kBinMaxHist)
                       ? (int)nb : 0;
  const bool one = n_atoms > 0 && n_atoms <= msm::kBinRowAtoms && own <= msm::kBinRowCells;
  g.bin_row_blocks = (one && !(P->prefer_bin2 && P->bin2_blocks > 0)) ? nbr : 0;
  g.bin_blocks = g.bin_row_blocks == 0 ? P->bin2_blocks : 0;
  // otherwise by cell row first, then within each row, when the rows fit the
  // row binning's LDS histograms (else four kernels over the cells)
  const bool by_rows = n_atoms > 0 && g.bin_row_blocks == 0 && g.bin_blocks == 0 && rows <= msm::kBinRowsMax;
  g.binr_blocks = by_rows ? (int)((n_atoms + msm::kBinRChunk - 1) / msm::kBinRChunk) : 0;
  set_row_items(g, g.item_chunks);
  set_short_blocks(g, P->short_cap);
}

// Cell reach of a new plan: finer rows (higher reach) cut the short-range
// candidates that fail the cutoff test, but a 64-atom chunk of a thin row
// spans a long stretch of x, so every work item stages more atoms (on the
// 1M-atom water box reach 4 doubled the short-range time); the autotuner
// tries the finer cells.
int default_reach(int) { return 2; }

void set_lattice_waves(msm_plan* P, int waves) {
  P->lat_waves = waves;
  if (P->lat.b > 0 && P->lat.waves != waves) {
    choose_lattice_tiles(P->g, P->rows_c, (int)P->weights.size(), P->lat.H, P->lat_tables, P->lat, P->lat.b, waves);
    refresh_launch(P);
  }
}

void retune(msm_plan* P, const msm_tuning& t) {
  if (t.cell_reach != 0 && t.cell_reach != P->g.reach) set_cell_geometry(P, t.cell_reach);
  if (t.lattice_b && P->lat.b && t.lattice_b != P->lat.b)
    choose_lattice_tiles(P->g, P->rows_c, (int)P->weights.size(), P->lat.H, P->lat_tables, P->lat,
                         t.lattice_b, P->lat_waves);
  Geom& g = P->g;
  if (t.item_chunks > 0) set_row_items(g, t.item_chunks);
  if (t.short_blocks != 0) P->short_cap = t.short_blocks < 0 ? 0 : t.short_blocks;
  if (t.streams != 0) P->streams = t.streams;
  if (t.short_after != 0) P->short_after = t.short_after;
  if (t.short_split != 0) P->short_split = t.short_split;
  set_short_blocks(g, P->short_cap);
  refresh_launch(P);
}

msm_status check_tuning(const msm_tuning* t) {
  if (!t) return fail(MSM_ERR_INVALID_ARG, "null tuning");
  if (t->lattice_b != 0 && t->lattice_b != 4 && t->lattice_b != 6 && t->lattice_b != 8)
    return fail(MSM_ERR_INVALID_ARG, "lattice_b must be 0, 4, 6 or 8");
  if (t->item_chunks < 0) return fail(MSM_ERR_INVALID_ARG, "item_chunks must be >= 0");
  if (t->short_blocks < -1) return fail(MSM_ERR_INVALID_ARG, "short_blocks must be >= -1");
  if (t->streams < 0 || t->streams > 3) return fail(MSM_ERR_INVALID_ARG, "streams must be 0 .. 3");
  if (t->short_after < 0 || t->short_after > 3) return fail(MSM_ERR_INVALID_ARG, "short_after must be 0 .. 3");
  if (t->short_split < 0 || t->short_split > 1000)
    return fail(MSM_ERR_INVALID_ARG, "short_split must be 0 .. 1000");
  if (t->cell_reach != 0 && (t->cell_reach < 2 || t->cell_reach > 4))
    return fail(MSM_ERR_INVALID_ARG, "cell_reach must be 0, 2, 3 or 4");
  if (t->reserved != 0) return fail(MSM_ERR_INVALID_ARG, "reserved tuning field must be zero");
  return MSM_OK;
}

hipError_t read_flags(const msm_plan* P, const char* ws, int32_t* flags) {
  int32_t w[msm::kStatusWords];
  const int nw = 64 + P->g.bin_row_blocks;
  hipError_t e = hipMemcpy(w, ws + P->lay.off[msm::kSecStatus], nw * sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  int32_t f = w[0];
  for (int b = 64; b < nw; ++b) f |= w[b];
  *flags = f;
  return hipSuccess;
}

msm::DevPtrs dev_ptrs(const msm_plan* P, void* ws) {
  char* b = static_cast<char*>(ws);
  const size_t* o = P->lay.off;
  msm::DevPtrs d;
  d.qgrid = (decltype(d.qgrid))(b + o[msm::kSecQGrid]);
  d.ucut = (decltype(d.ucut))(b + o[msm::kSecUCut]);
  d.u = (decltype(d.u))(b + o[msm::kSecU]);
  d.sorted = (decltype(d.sorted))(b + o[msm::kSecSorted]);
  d.perm = (decltype(d.perm))(b + o[msm::kSecPerm]);
  d.fshort = (decltype(d.fshort))(b + o[msm::kSecShort]);
  d.status = (decltype(d.status))(b + o[msm::kSecStatus]);
  d.counts = (decltype(d.counts))(b + o[msm::kSecCounts]);
  d.cell_start = (decltype(d.cell_start))(b + o[msm::kSecCellStart]);
  d.cursor = (decltype(d.cursor))(b + o[msm::kSecCursor]);
  d.cell_of = (decltype(d.cell_of))(b + o[msm::kSecCellOf]);
  d.tmp = (decltype(d.tmp))(b + o[msm::kSecTmp]);
  d.bin_hist = (decltype(d.bin_hist))(b + o[msm::kSecBinHist]);
  d.scan = (decltype(d.scan))(b + o[msm::kSecScan]);
  d.ant_part = (decltype(d.ant_part))(b + o[msm::kSecAntPart]);
  d.rows = (decltype(d.rows))(b + o[msm::kSecRows]);
  d.weights = (decltype(d.weights))(b + o[msm::kSecWeights]);
  d.rows_c = (decltype(d.rows_c))(b + o[msm::kSecRowsC]);
  d.weights_c = (decltype(d.weights_c))(b + o[msm::kSecWeightsC]);
  d.top = (decltype(d.top))(b + o[msm::kSecTop]);
  d.partials = (decltype(d.partials))(b + o[msm::kSecPartials]);
  d.lat_part = (decltype(d.lat_part))(b + o[msm::kSecLatPart]);
  d.excl_start = (decltype(d.excl_start))(P->excl_start);
  d.excl_idx = (decltype(d.excl_idx))(P->excl_idx);
  d.excl_nnz = P->excl_nnz;
  return d;
}

extern "C" {

const char* msm_status_string(msm_status s) {
  switch (s) {
    case MSM_OK: return "ok";
    case MSM_ERR_INVALID_ARG: return "invalid argument";
    case MSM_ERR_OUT_OF_BOX: return "atom outside the box";
    case MSM_ERR_NONFINITE: return "non-finite position or charge";
    case MSM_ERR_WORKSPACE: return "workspace missing or too small";
    case MSM_ERR_HIP: return "HIP runtime error";
    case MSM_ERR_UNSUPPORTED: return "unsupported configuration";
    case MSM_ERR_COINCIDENT: return "coincident atoms";
  }
  return "unknown status";
}

const char* msm_last_error(void) { return g_last_error.c_str(); }

msm_status msm_plan_create(const msm_params* prm, int32_t n_atoms, msm_plan** out) {
  if (!prm || !out) return fail(MSM_ERR_INVALID_ARG, "null params or output pointer");
  *out = nullptr;
  const msm_params& p = *prm;
  if (!finite_pos(p.cutoff)) return fail(MSM_ERR_INVALID_ARG, "cutoff must be finite and > 0");
  if (!finite_pos(p.spacing)) return fail(MSM_ERR_INVALID_ARG, "spacing must be finite and > 0");
  if (p.order != 4 && p.order != 6) return fail(MSM_ERR_INVALID_ARG, "order must be 4 or 6");
  if (p.split_m < 0 || p.split_m > 7) return fail(MSM_ERR_INVALID_ARG, "split_m must be in [0, 7]");
  if (p.levels < 0 || p.levels > msm::kMaxLevels)
    return fail(MSM_ERR_INVALID_ARG, "levels must be in [0, 12]");
  if (p.periodic != 0 && p.periodic != 1) return fail(MSM_ERR_INVALID_ARG, "periodic must be 0 or 1");
  if (n_atoms < 0) return fail(MSM_ERR_INVALID_ARG, "n_atoms must be >= 0");
  if (!std::isfinite(p.coulomb_k)) return fail(MSM_ERR_INVALID_ARG, "coulomb_k must be finite");
  for (int d = 0; d < 3; ++d) {
    if (!finite_pos(p.box_len[d])) return fail(MSM_ERR_INVALID_ARG, "box_len must be finite and > 0");
    if (!std::isfinite(p.box_lo[d])) return fail(MSM_ERR_INVALID_ARG, "box_lo must be finite");
  }
  // periodic grids: a whole number of nodes per period, halving at every level
  int per0[3] = {0, 0, 0};
  if (p.periodic) {
    for (int d = 0; d < 3; ++d) {
      const double t = p.box_len[d] / p.spacing;
      const double r = std::nearbyint(t);
      if (r < 1.0 || r > 1.0e6 || std::fabs(t - r) > 1e-9 * t)
        return fail(MSM_ERR_INVALID_ARG, "periodic: box_len / spacing must be an integer (at most 1e6)");
      if (2.0 * p.cutoff > p.box_len[d]) return fail(MSM_ERR_INVALID_ARG, "periodic: 2 cutoff must not exceed box_len");
      per0[d] = (int)r;
    }
  }

  msm_plan* P = new (std::nothrow) msm_plan();
  if (!P) return fail(MSM_ERR_INVALID_ARG, "out of host memory");
  static std::atomic<uint64_t> next_uid{1};
  P->uid = next_uid.fetch_add(1);
  P->p = p;
  Geom& g = P->g;
  std::memset(&g, 0, sizeof(g));
  const double a = p.cutoff, h = p.spacing;
  g.n_atoms = n_atoms;
  g.order = p.order;
  g.half = p.order / 2;
  g.h = (float)h;
  g.inv_h = (float)(1.0 / h);
  g.m = p.split_m ? p.split_m : p.order / 2;
  g.ke = p.coulomb_k != 0.0 ? p.coulomb_k : 1.0;
  double maxlen = 0.0;
  g.periodic = p.periodic;
  for (int d = 0; d < 3; ++d) {
    g.lo[d] = p.box_lo[d];
    g.hi[d] = p.box_lo[d] + p.box_len[d];
    g.lo_f[d] = (float)p.box_lo[d];
    g.len_f[d] = (float)p.box_len[d];
    g.len[d] = p.box_len[d];
    g.inv_len_f[d] = (float)(1.0 / p.box_len[d]);
    double fm = p.periodic ? (double)per0[d] : std::floor(p.box_len[d] / h);
    if (fm > 1.0e6) {
      delete P;
      return fail(MSM_ERR_UNSUPPORTED, "grid too fine for the box (more than 1e6 nodes per side)");
    }
    g.fmax[d] = (int)fm;
    maxlen = std::max(maxlen, p.box_len[d]);
  }

  // levels: given, or the fewest whose top interior spans <= 8 nodes per side
  // (periodic: whose top grid has <= 8 nodes per side, as far as the levels halve)
  int L = p.levels;
  if (L == 0 && p.periodic) {
    L = 1;
    for (;;) {
      bool big = false, even = true;
      for (int d = 0; d < 3; ++d) {
        big = big || (per0[d] >> (L - 1)) > 8;
        even = even && (per0[d] >> (L - 1)) % 2 == 0;
      }
      if (!big || !even || L == msm::kMaxLevels) break;
      ++L;
    }
  } else if (L == 0) {
    L = msm::kMaxLevels;
    for (int l = 1; l <= msm::kMaxLevels; ++l)
      if ((int)std::ceil(maxlen / std::ldexp(h, l - 1)) + 1 <= 8) {
        L = l;
        break;
      }
  }
  if (p.periodic)
    for (int d = 0; d < 3; ++d)
      if (per0[d] % (1 << (L - 1))) {
        delete P;
        return fail(MSM_ERR_INVALID_ARG, "periodic: box_len / spacing must be divisible by 2^(levels-1)");
      }
  g.levels = L;
  // periodic: level k holds its per0 / 2^k nodes of one period with ghost
  // copies on each side, as many as the widest stencil reaching past a period
  // needs (lattice half-width, restriction reach order - 1, basis support)
  if (p.periodic) {
    int H = 0;
    if (L > 1)
      while ((H + 1) * h < 2.0 * a) ++H;
    g.ghost = std::max({H, p.order - 1, g.half + 1});
  }
  // level 0 spans the nodes atoms in the box touch; level k+1 the nodes level k restricts to
  long long off = 0;
  for (int k = 0; k < L; ++k) {
    msm::Level& lv = g.lv[k];
    for (int d = 0; d < 3; ++d) {
      int lo, hi;
      if (p.periodic) {
        lv.per[d] = per0[d] >> k;
        lo = -g.ghost;
        hi = lv.per[d] - 1 + g.ghost;
      } else if (k == 0) {
        lo = -(g.half - 1);
        hi = g.fmax[d] + g.half;
      } else {
        const msm::Level& pv = g.lv[k - 1];
        lo = ceil_div2(pv.lo[d] - (p.order - 1));
        hi = floor_div2(pv.lo[d] + pv.n[d] - 1 + (p.order - 1));
      }
      lv.lo[d] = lo;
      lv.n[d] = hi - lo + 1;
    }
    long long cnt = (long long)lv.n[0] * lv.n[1] * lv.n[2];
    if (off + cnt > (1LL << 28)) {
      delete P;
      return fail(MSM_ERR_UNSUPPORTED, "grid hierarchy exceeds 2^28 nodes");
    }
    lv.off = (int)off;
    lv.count = (int)cnt;
    off += cnt;
  }
  g.total_nodes = (int)off;
  if (g.lv[L - 1].count > msm::kMaxTopNodes) {
    delete P;
    return fail(MSM_ERR_UNSUPPORTED, "top level too large for the all-pairs sum; use more levels");
  }

  // anterpolation tiles: start from 16 x 16 x 8 level-0 nodes and halve the
  // largest side (down to 1) until there are at least 512 tiles, so a launch
  // covers the 256 compute units twice (a coarse grid, e.g. h = 10 A, has few
  // nodes but as many atoms: its tiles shrink to a few nodes each)
  {
    int t[3] = {16, 16, 8};
    auto tiles = [&]() {
      long long n = 1;
      for (int d = 0; d < 3; ++d) n *= (g.fmax[d] + t[d]) / t[d];
      return n;
    };
    while (tiles() < 512) {
      int d = 0;
      for (int e = 1; e < 3; ++e)
        if (t[e] > t[d]) d = e;
      if (t[d] <= 1) break;
      t[d] /= 2;
    }
    g.at_ext = 1;
    for (int d = 0; d < 3; ++d) {
      g.at[d] = t[d];
      g.atn[d] = (g.fmax[d] + t[d]) / t[d];          // tiles covering floor indices 0 .. fmax
      g.at_ext *= t[d] + p.order - 1;
    }
  }

  // smoothing constants
  double c[9];
  taylor_coeffs(g.m, c);
  for (int k = 0; k <= g.m; ++k) {
    g.dr[k] = (float)(2.0 * k * c[k] / std::pow(a, 2.0 * k + 1.0));
  }
  g.self = (float)(c[0] / a);
  g.inv_a = (float)(1.0 / a);
  g.inv_a2f = (float)(1.0 / (a * a));
  g.a2 = (float)(a * a);
  g.inv_a2 = (float)(1.0 / (a * a));

  // link cells: the finest reach any tuning may ask for sizes the cell
  // sections; the plan starts at the default reach
  g.a_win = (float)(a * (1.0 + 1e-4));
  g.item_chunks = 1;
  for (int r : {2, 3, 4}) {
    set_cell_geometry(P, r);
    P->max_cells = std::max(P->max_cells, g.n_cells);
    P->max_bin_hist = std::max(P->max_bin_hist, (long long)P->bin2_blocks * ((g.n_cells + 3) & ~3));
  }
  g.max_cells = P->max_cells;
  set_cell_geometry(P, default_reach(n_atoms));

  // lattice-cutoff stencil: W(n) = g^0(h |n|) for h |n| < 2a, rows along z
  if (L > 1) {
    const double rad = 2.0 * a / h;
    if (rad > 48.0) {
      delete P;
      return fail(MSM_ERR_UNSUPPORTED, "stencil radius 2a/h above 48 nodes");
    }
    int Rn = (int)std::ceil(rad);
    for (int nx = -Rn; nx <= Rn; ++nx)
      for (int ny = -Rn; ny <= Rn; ++ny) {
        int zr = -1;
        for (int nz = 0; nz <= Rn; ++nz) {
          double dist = h * std::sqrt((double)(nx * nx + ny * ny + nz * nz));
          if (dist < 2.0 * a) zr = nz;
        }
        if (zr < 0) continue;
        msm::StencilRow row{nx, ny, zr, (int)P->weights.size()};
        for (int nz = -zr; nz <= zr; ++nz) {
          double dist = h * std::sqrt((double)(nx * nx + ny * ny + nz * nz));
          double w0 = gamma_h(c, g.m, dist / a) / a - gamma_h(c, g.m, dist / (2.0 * a)) / (2.0 * a);
          P->weights.push_back((float)w0);
        }
        P->rows.push_back(row);
      }
  }
  // compact stencil for the windowed kernel: for |nz|, ny >= 0 the weights
  // W(nx) for nx = 0..xr (padded to a multiple of 4); rows for nz in [-H, H]
  if (L > 1) {
    int H = 0;
    for (const auto& r : P->rows) H = std::max(H, std::abs(r.nx));
    if (H <= msm::kLatMaxHalo) {
      auto xrow = [&](int az, int ay) {
        int xr = -1;
        for (int nx = 0; nx <= H; ++nx)
          if (h * std::sqrt((double)(nx * nx + ay * ay + az * az)) < 2.0 * a) xr = nx;
        return xr;
      };
      std::vector<int> woff((size_t)(H + 1) * (H + 1), -1);
      for (int az = 0; az <= H; ++az)
        for (int ay = 0; ay <= H; ++ay) {
          const int xr = xrow(az, ay);
          if (xr < 0) continue;
          woff[(size_t)az * (H + 1) + ay] = (int)P->weights_c.size();
          for (int nx = 0; nx <= xr; ++nx) {
            const double dist = h * std::sqrt((double)(nx * nx + ay * ay + az * az));
            P->weights_c.push_back((float)(gamma_h(c, g.m, dist / a) / a -
                                           gamma_h(c, g.m, dist / (2.0 * a)) / (2.0 * a)));
          }
          while (P->weights_c.size() % 4) P->weights_c.push_back(0.f);
        }
      for (int nz = -H; nz <= H; ++nz)
        for (int ay = 0; ay <= H; ++ay) {
          const int az = std::abs(nz);
          const int xr = xrow(az, ay);
          if (xr >= 0) P->rows_c.push_back(make_int4(nz, ay, xr, woff[(size_t)az * (H + 1) + ay]));
        }
      P->lat.n_rows = (int)P->rows_c.size();
      P->lat.n_wc = (int)P->weights_c.size();
      const int tables = P->lat.n_rows * 16 + P->lat.n_wc * 4;
      P->lat_tables = tables;
      // the partials section holds the largest need of any tuning
      for (int b : {4, 6, 8})
        for (int w : {msm::kLatWavesFew, msm::kLatWavesMany}) {
          choose_lattice_tiles(g, P->rows_c, (int)P->weights.size(), H, tables, P->lat, b, w);
          P->lat_part_max = std::max(P->lat_part_max, P->lat.n_part);
        }
      choose_lattice_tiles(g, P->rows_c, (int)P->weights.size(), H, tables, P->lat, 0, P->lat_waves);
    } else {
      P->lat.b = 0;
      P->lat.H = H;
    }
  }
  // top level (float64): T(d) = g^{l-1}(2^{l-1} h |d|) = gamma(r / A) / A, A = 2^{l-1} a
  // (periodic: the image sum K(d) over the node offsets of one period)
  if (p.periodic) {
    const msm::Level& T = g.lv[L - 1];
    periodic_top_table(c, g.m, std::ldexp(a, L - 1), std::ldexp(h, L - 1), T.per, p.box_len, P->top);
  } else {
    const msm::Level& T = g.lv[L - 1];
    const double A = std::ldexp(a, L - 1), hk = std::ldexp(h, L - 1);
    P->top.resize((size_t)T.count);
    for (int dz = 0; dz < T.n[2]; ++dz)
      for (int dy = 0; dy < T.n[1]; ++dy)
        for (int dx = 0; dx < T.n[0]; ++dx) {
          double r = hk * std::sqrt((double)(dx * dx + dy * dy + dz * dz));
          P->top[((size_t)dz * T.n[1] + dy) * T.n[0] + dx] = gamma_h(c, g.m, r / A) / A;
        }
  }
  P->n_partials = msm::interp_partials(g);

  // workspace layout
  Layout& lay = P->lay;
  size_t n = (size_t)std::max(n_atoms, 1);
  size_t nodes = (size_t)g.total_nodes;
  lay.bytes[msm::kSecQGrid] = nodes * sizeof(float);
  lay.bytes[msm::kSecUCut] = nodes * sizeof(float);
  lay.bytes[msm::kSecU] = nodes * sizeof(float);
  lay.bytes[msm::kSecSorted] = n * sizeof(float4);
  lay.bytes[msm::kSecPerm] = n * sizeof(int);
  lay.bytes[msm::kSecShort] = n * sizeof(float4);
  lay.bytes[msm::kSecStatus] = msm::kStatusWords * sizeof(int);
  lay.bytes[msm::kSecCounts] = ((size_t)P->max_cells + 1) * sizeof(int);
  lay.bytes[msm::kSecCellStart] = ((size_t)P->max_cells + 1) * sizeof(int);
  lay.bytes[msm::kSecCursor] = (size_t)P->max_cells * sizeof(int);
  lay.bytes[msm::kSecCellOf] = n * sizeof(int);
  lay.bytes[msm::kSecTmp] = n * sizeof(int);
  // sized for the two-kernel binning wherever it is possible (a batch may
  // switch a system to it)
  lay.bytes[msm::kSecBinHist] = std::max<size_t>((size_t)P->max_bin_hist, 1) * sizeof(int);
  // tile totals of the four-kernel binning's scan, or the row starts of the row binning
  lay.bytes[msm::kSecScan] = ((size_t)P->max_cells + 1) * sizeof(int);
  lay.bytes[msm::kSecAntPart] = (size_t)g.atn[0] * g.atn[1] * g.atn[2] * g.at_ext * sizeof(long long);
  lay.bytes[msm::kSecRows] = std::max<size_t>(P->rows.size(), 1) * sizeof(msm::StencilRow);
  lay.bytes[msm::kSecWeights] = std::max<size_t>(P->weights.size(), 1) * sizeof(float);
  lay.bytes[msm::kSecRowsC] = std::max<size_t>(P->rows_c.size(), 1) * sizeof(int4);
  lay.bytes[msm::kSecWeightsC] = std::max<size_t>(P->weights_c.size(), 1) * sizeof(float);
  lay.bytes[msm::kSecTop] = P->top.size() * sizeof(double);
  lay.bytes[msm::kSecPartials] = 10 * (size_t)P->n_partials * sizeof(double);
  lay.bytes[msm::kSecLatPart] = std::max<size_t>(P->lat_part_max, 1) * sizeof(double);
  lay.bytes[msm::kSecDesc] = sizeof(msm::SysDesc);
  size_t o = 0;
  for (int s = 0; s < msm::kSecCount; ++s) {
    lay.off[s] = o;
    o += align256(lay.bytes[s]);
  }
  lay.total = o;

  refresh_launch(P);
  *out = P;
  return MSM_OK;
}

msm_status msm_pair_plan_create(const msm_pair_params* pp, int32_t n_atoms, msm_plan** out) {
  if (!pp || !out) return fail(MSM_ERR_INVALID_ARG, "null params or output pointer");
  *out = nullptr;
  if (pp->kind < MSM_PAIR_CUTOFF || pp->kind > MSM_PAIR_WOLF)
    return fail(MSM_ERR_INVALID_ARG, "kind must be MSM_PAIR_CUTOFF, MSM_PAIR_SHIFTED_FORCE or MSM_PAIR_WOLF");
  if (pp->periodic != 0 && pp->periodic != 1) return fail(MSM_ERR_INVALID_ARG, "periodic must be 0 or 1");
  if (!finite_pos(pp->cutoff)) return fail(MSM_ERR_INVALID_ARG, "cutoff must be finite and > 0");
  for (int d = 0; d < 3; ++d)
    if (pp->periodic && finite_pos(pp->box_len[d]) && 2.0 * pp->cutoff > pp->box_len[d])
      return fail(MSM_ERR_INVALID_ARG, "periodic: 2 cutoff must not exceed box_len");
  if (!std::isfinite(pp->alpha) || pp->alpha < 0.0) return fail(MSM_ERR_INVALID_ARG, "alpha must be finite and >= 0");
  // the cells, binning and short-range pass of an MSM plan with cutoff rc; its
  // (unused) grid is one coarse level
  msm_params p{};
  p.cutoff = pp->cutoff;
  double maxlen = 0.0;
  for (int d = 0; d < 3; ++d) {
    p.box_lo[d] = pp->box_lo[d];
    p.box_len[d] = pp->box_len[d];
    if (std::isfinite(pp->box_len[d])) maxlen = std::max(maxlen, pp->box_len[d]);
  }
  p.spacing = std::max(pp->cutoff, maxlen / 8.0);
  p.order = 4;
  p.levels = 1;
  p.coulomb_k = pp->coulomb_k;
  msm_plan* P = nullptr;
  msm_status st = msm_plan_create(&p, n_atoms, &P);
  if (st != MSM_OK) return st;
  Geom& g = P->g;
  const double rc = pp->cutoff, al = pp->alpha;
  g.pair = pp->kind;
  g.periodic = pp->periodic;                     // pairs at their nearest image (the grid is unused)
  assign_short_rows(g);                          // periodic plans walk rows one at a time
  g.pk[0] = g.pk[1] = g.pk[2] = g.pk[3] = 0.f;
  g.self = 0.f;
  if (pp->kind == MSM_PAIR_SHIFTED_FORCE) {
    g.pk[0] = (float)(1.0 / rc);
    g.pk[1] = (float)(1.0 / (rc * rc));
  } else if (pp->kind == MSM_PAIR_WOLF) {
    const double two_over_sqrt_pi = 1.1283791670955126;
    g.pk[0] = (float)al;
    g.pk[1] = (float)(std::erfc(al * rc) / rc);
    g.pk[2] = (float)(al * two_over_sqrt_pi);
    g.pk[3] = (float)(-al * al * 1.4426950408889634);   // -alpha^2 log2(e)
    // every pair the device evaluates has alpha r <= alpha rc (the r < rc test,
    // with float rounding to spare); below x = 1 the fit is as good and beyond
    // x = 10 erfc(x) exp(-x^2) underflows float
    const double x_hi = std::min(std::max(al * rc * (1.0 + 1e-3), 1.0), 10.0);
    if (fit_wolf_erfc(x_hi, g.ec) > 1e-7) {
      msm_plan_destroy(P);
      return fail(MSM_ERR_UNSUPPORTED, "Wolf erfc fit failed");
    }
    // phi_i gains 2 s q_i with s = -(erfc(alpha rc)/(2 rc) + alpha/sqrt(pi)); the
    // assembly subtracts q_i self
    g.self = (float)(std::erfc(al * rc) / rc + al * two_over_sqrt_pi);
  }
  P->pp = *pp;
  refresh_launch(P);
  *out = P;
  return MSM_OK;
}

msm_status msm_plan_destroy(msm_plan* plan) {
  if (plan) {
    for (auto& e : plan->ev)
      if (e) (void)hipEventDestroy(e);
    destroy_aux(plan->aux);
  }
  delete plan;
  return MSM_OK;
}

msm_status msm_profile_enable(msm_plan* P, int32_t enable) {
  if (!P) return fail(MSM_ERR_INVALID_ARG, "null plan");
  if (enable < 0 || enable > 2) return fail(MSM_ERR_INVALID_ARG, "profile mode must be 0, 1 or 2");
  if (enable && !P->ev[0])
    for (auto& e : P->ev) {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return hip_fail(r, "create timing events");
    }
  P->profile = enable;
  P->profiled = false;
  return MSM_OK;
}

msm_status msm_profile_read(const msm_plan* P, float* ms, int32_t* n_stages) {
  if (!P || !ms || !n_stages) return fail(MSM_ERR_INVALID_ARG, "null argument");
  if (!P->profile) return fail(MSM_ERR_INVALID_ARG, "profiling is not enabled on this plan");
  if (!P->profiled) return fail(MSM_ERR_INVALID_ARG, "no evaluation was timed since profiling was enabled");
  hipError_t r;
  if (P->profile == 1) {
    r = hipEventSynchronize(P->ev[msm::kStageCount]);
    if (r != hipSuccess) return hip_fail(r, "wait for timing events");
    for (int i = 0; i < msm::kStageCount; ++i) {
      r = hipEventElapsedTime(&ms[i], P->ev[i], P->ev[i + 1]);
      if (r != hipSuccess) return hip_fail(r, "read timing events");
    }
  } else {
    float slot[msm::kLiveSlots];
    for (int i = 0; i < msm::kLiveSlots; ++i) {
      r = hipEventSynchronize(P->ev[msm::kLiveSlots + i]);
      if (r == hipSuccess) r = hipEventElapsedTime(&slot[i], P->ev[i], P->ev[msm::kLiveSlots + i]);
      if (r != hipSuccess) return hip_fail(r, "read timing events");
    }
    for (int i = 0; i < msm::kStageCount; ++i) ms[i] = slot[i];
    ms[msm::kStageShort] += slot[msm::kSlotShort2];
    ms[msm::kStageLattice] += slot[msm::kSlotLattice0];
  }
  *n_stages = msm::kStageCount;
  return MSM_OK;
}

msm_status msm_plan_info(const msm_plan* P, int32_t* levels, int32_t* grid_lo, int32_t* grid_n) {
  if (!P || !levels) return fail(MSM_ERR_INVALID_ARG, "null plan or levels pointer");
  *levels = P->g.levels;
  for (int k = 0; k < P->g.levels; ++k)
    for (int d = 0; d < 3; ++d) {
      if (grid_lo) grid_lo[3 * k + d] = P->g.lv[k].lo[d];
      if (grid_n) grid_n[3 * k + d] = P->g.lv[k].n[d];
    }
  return MSM_OK;
}

msm_status msm_plan_describe(const msm_plan* P, char* buf, size_t buf_bytes) {
  if (!P || !buf || buf_bytes == 0) return fail(MSM_ERR_INVALID_ARG, "null plan or buffer");
  const Geom& g = P->g;
  std::string o = "{";
  o += "\"pair\": " + std::to_string(g.pair) + ", \"levels\": " + std::to_string(g.levels);
  o += ", \"cells\": [" + std::to_string(g.nc[0]) + ", " + std::to_string(g.nc[1]) + ", " +
       std::to_string(g.nc[2]) + "], \"reach\": " + std::to_string(g.reach) +
       ", \"bin_blocks\": " + std::to_string(g.bin_blocks) +
       ", \"bin_row_blocks\": " + std::to_string(g.bin_row_blocks) + ", \"binr_blocks\": " +
       std::to_string(g.binr_blocks) +
       ", \"item_chunks\": " + std::to_string(g.item_chunks) + ", \"short_blocks\": " + std::to_string(g.short_blocks) +
       ", \"streams\": " + std::to_string(P->streams) + ", \"short_after\": " + std::to_string(P->short_after) +
       ", \"short_split\": " + std::to_string(P->short_split);
  o += ", \"taps\": " + std::to_string(P->weights.size()) + ", \"halo\": " + std::to_string(P->lat.H);
  o += ", \"lattice_b\": " + std::to_string(P->lat.b) + ", \"lattice_waves\": " + std::to_string(P->lat.waves) +
       ", \"lattice_lds\": " +
       std::to_string(P->lat.lds_bytes) + ", \"lattice_tiles\": [";
  for (int k = 0; k < P->lat.n; ++k) {
    const msm::LatTile& t = P->lat.t[k];
    if (k) o += ", ";
    o += "[" + std::to_string(t.xl) + ", " + std::to_string(t.ty) + ", " + std::to_string(t.tz) + ", " +
         std::to_string(t.ntx * t.nty * t.ntz) + ", " +
         std::to_string(bank_conflicts(t.xl, t.ty, t.tz, P->lat.b, t.px, t.pp)) + ", " +
         std::to_string(t.groups) + "]";
  }
  o += "], \"prolong_per_level\": " + std::to_string(P->lg.prolong_split ? 1 : 0);
  o += ", \"periodic\": " + std::to_string(g.periodic) + ", \"ghost\": " + std::to_string(g.ghost);
  o += ", \"workspace_bytes\": " + std::to_string(P->lay.total) + "}";
  std::strncpy(buf, o.c_str(), buf_bytes - 1);
  buf[buf_bytes - 1] = 0;
  return o.size() < buf_bytes ? MSM_OK : fail(MSM_ERR_INVALID_ARG, "buffer too small");
}

msm_status msm_workspace_bytes(const msm_plan* P, size_t* bytes) {
  if (!P || !bytes) return fail(MSM_ERR_INVALID_ARG, "null plan or bytes pointer");
  *bytes = P->lay.total;
  return MSM_OK;
}

msm_status msm_workspace_section(const msm_plan* P, int32_t section, size_t* offset, size_t* bytes) {
  if (!P || section < 0 || section > msm::kSecShort)
    return fail(MSM_ERR_INVALID_ARG, "null plan or unknown section");
  if (offset) *offset = P->lay.off[section];
  if (bytes) *bytes = P->lay.bytes[section];
  return MSM_OK;
}


}  // extern "C"

// Upload the plan's tables and descriptor into the workspace at ws (device)
// and clear its cell counters, on stream s; waits for the copies (they read
// pageable host memory of the plan).
msm_status init_workspace(const msm_plan* P, void* ws, hipStream_t s) {
  char* base = static_cast<char*>(ws);
  hipError_t e;
  if (!P->rows.empty()) {
    e = hipMemcpyAsync(base + P->lay.off[msm::kSecRows], P->rows.data(),
                       P->rows.size() * sizeof(msm::StencilRow), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "upload stencil rows");
    e = hipMemcpyAsync(base + P->lay.off[msm::kSecWeights], P->weights.data(),
                       P->weights.size() * sizeof(float), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "upload stencil weights");
    if (!P->rows_c.empty()) {
      e = hipMemcpyAsync(base + P->lay.off[msm::kSecRowsC], P->rows_c.data(),
                         P->rows_c.size() * sizeof(int4), hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return hip_fail(e, "upload compact stencil rows");
      e = hipMemcpyAsync(base + P->lay.off[msm::kSecWeightsC], P->weights_c.data(),
                         P->weights_c.size() * sizeof(float), hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return hip_fail(e, "upload compact stencil weights");
    }
  }
  e = hipMemcpyAsync(base + P->lay.off[msm::kSecTop], P->top.data(), P->top.size() * sizeof(double),
                     hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "upload top-level table");
  msm_plan* M = const_cast<msm_plan*>(P);
  M->desc.d = dev_ptrs(P, ws);
  e = hipMemcpyAsync(base + P->lay.off[msm::kSecDesc], &M->desc, sizeof(msm::SysDesc),
                     hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "upload descriptor");
  msm::LaunchGeom L = P->lg;
  L.sys = reinterpret_cast<const msm::SysDesc*>(base + P->lay.off[msm::kSecDesc]);
  e = msm::launch_init(L, s);
  if (e != hipSuccess) return hip_fail(e, "clear cell counters");
  // pageable-memory copies are staged before returning; the plan may be destroyed afterwards
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "workspace init");
  return MSM_OK;
}

extern "C" {

msm_status msm_workspace_init(const msm_plan* P, void* ws, size_t ws_bytes, msm_stream_t stream) {
  if (!P) return fail(MSM_ERR_INVALID_ARG, "null plan");
  if (!ws || ws_bytes < P->lay.total) return fail(MSM_ERR_WORKSPACE, "workspace missing or too small");
  const msm_status st = init_workspace(P, ws, reinterpret_cast<hipStream_t>(stream));
  if (st != MSM_OK) return st;
  const_cast<msm_plan*>(P)->ready.insert(ws);
  return MSM_OK;
}


static msm::LaunchGeom launch_geom(const msm_plan* P, void* ws) {
  msm::LaunchGeom L = P->lg;
  L.sys = reinterpret_cast<const msm::SysDesc*>(static_cast<char*>(ws) + P->lay.off[msm::kSecDesc]);
  return L;
}

static msm_status check_call(const msm_plan* P, const void* ws, size_t ws_bytes, const float* x,
                             const float* y, const float* z, const float* q, const float* fx,
                             const float* fy, const float* fz) {
  if (!P) return fail(MSM_ERR_INVALID_ARG, "null plan");
  if (!ws || ws_bytes < P->lay.total) return fail(MSM_ERR_WORKSPACE, "workspace missing or too small");
  if (!P->ready.count(ws)) return fail(MSM_ERR_WORKSPACE, "workspace not initialised for this plan");
  if (P->g.n_atoms > 0 && (!x || !y || !z || !q))
    return fail(MSM_ERR_INVALID_ARG, "null position or charge array");
  if (!((fx && fy && fz) || (!fx && !fy && !fz)))
    return fail(MSM_ERR_INVALID_ARG, "vector outputs must be all set or all null");
  return MSM_OK;
}

msm_status msm_compute(const msm_plan* P, void* ws, size_t ws_bytes, msm_stream_t stream,
                       const float* x, const float* y, const float* z, const float* q, float* fx,
                       float* fy, float* fz, float* phi, double* energy, double* virial) {
  msm_status st = check_call(P, ws, ws_bytes, x, y, z, q, fx, fy, fz);
  if (st != MSM_OK) return st;
  msm_plan* M = const_cast<msm_plan*>(P);
  hipError_t e = ensure_aux(M->aux);
  if (e != hipSuccess) return hip_fail(e, "create auxiliary stream");
  const msm::Io io{x, y, z, q, fx, fy, fz, phi, energy, virial, nullptr};
  e = msm::launch_eval(msm::kModeForces, launch_geom(P, ws), reinterpret_cast<hipStream_t>(stream), io,
                       P->profile ? M->ev : nullptr, &M->aux.cc, P->profile == 2);
  if (P->profile) M->profiled = true;
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return MSM_OK;
}

static msm_status eval_mode(int mode, const msm_plan* P, void* ws, size_t ws_bytes,
                            msm_stream_t stream, const float* x, const float* y, const float* z,
                            const float* q, float* fx, float* fy, float* fz, float* phi,
                            double* energy, const double* gscale) {
  msm_status st = check_call(P, ws, ws_bytes, x, y, z, q, fx, fy, fz);
  if (st != MSM_OK) return st;
  msm_plan* M = const_cast<msm_plan*>(P);
  hipError_t e = ensure_aux(M->aux);
  if (e != hipSuccess) return hip_fail(e, "create auxiliary stream");
  const msm::Io io{x, y, z, q, fx, fy, fz, phi, energy, nullptr, gscale};
  e = msm::launch_eval(mode, launch_geom(P, ws), reinterpret_cast<hipStream_t>(stream), io, nullptr,
                       &M->aux.cc);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return MSM_OK;
}

msm_status msm_energy(const msm_plan* P, void* ws, size_t ws_bytes, msm_stream_t stream,
                      const float* x, const float* y, const float* z, const float* q,
                      double* energy) {
  if (!energy) return fail(MSM_ERR_INVALID_ARG, "null energy output");
  if (P && P->g.pair) return fail(MSM_ERR_UNSUPPORTED, "msm_energy is for multilevel-summation plans");
  return eval_mode(msm::kModeEnergy, P, ws, ws_bytes, stream, x, y, z, q, nullptr, nullptr, nullptr,
                   nullptr, energy, nullptr);
}

msm_status msm_backward(const msm_plan* P, void* ws, size_t ws_bytes, msm_stream_t stream,
                        const float* x, const float* y, const float* z, const float* q,
                        const double* grad_energy, float* dedx, float* dedy, float* dedz,
                        float* dedq) {
  if (!grad_energy) return fail(MSM_ERR_INVALID_ARG, "null grad_energy");
  if (P && P->g.pair) return fail(MSM_ERR_UNSUPPORTED, "msm_backward is for multilevel-summation plans");
  return eval_mode(msm::kModeGradient, P, ws, ws_bytes, stream, x, y, z, q, dedx, dedy, dedz, dedq,
                   nullptr, grad_energy);
}

msm_status msm_graph_destroy(msm_graph* G) {
  if (G) {
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
  }
  return MSM_OK;
}

msm_status msm_graph_capture(const msm_plan* P, void* ws, size_t ws_bytes, const float* x,
                             const float* y, const float* z, const float* q, float* fx, float* fy,
                             float* fz, float* phi, double* energy, double* virial, msm_graph** out) {
  if (!out) return fail(MSM_ERR_INVALID_ARG, "null output pointer");
  *out = nullptr;
  msm_status st = check_call(P, ws, ws_bytes, x, y, z, q, fx, fy, fz);
  if (st != MSM_OK) return st;
  msm_plan* M = const_cast<msm_plan*>(P);
  hipError_t e = ensure_aux(M->aux);
  if (e != hipSuccess) return hip_fail(e, "create auxiliary stream");
  const msm::Io io{x, y, z, q, fx, fy, fz, phi, energy, virial, nullptr};
  const msm::LaunchGeom L = launch_geom(P, ws);
  return capture_graph(
      [&](hipStream_t cs) {
        return msm::launch_eval(msm::kModeForces, L, cs, io, nullptr, &M->aux.cc);
      },
      &M->tune_gen, out);
}

msm_status msm_graph_launch(const msm_graph* G, msm_stream_t stream) {
  if (!G || !G->exec) return fail(MSM_ERR_INVALID_ARG, "null graph");
  if (G->owner_gen && *G->owner_gen != G->gen)
    return fail(MSM_ERR_INVALID_ARG, "the plan or batch was re-tuned after this graph was captured");
  hipError_t e = hipGraphLaunch(G->exec, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return MSM_OK;
}

msm_status msm_status_query(const msm_plan* P, const void* ws, msm_stream_t stream,
                            int32_t* device_flags) {
  if (!P || !ws) return fail(MSM_ERR_INVALID_ARG, "null plan or workspace");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  int32_t flags = 0;
  e = read_flags(P, static_cast<const char*>(ws), &flags);
  if (e != hipSuccess) return hip_fail(e, "read status");
  if (device_flags) *device_flags = flags;
  if (flags & msm::kFlagNonFinite) return fail(MSM_ERR_NONFINITE, "non-finite position or charge");
  if (flags & msm::kFlagOutOfBox) return fail(MSM_ERR_OUT_OF_BOX, "atom outside the box");
  if (flags & msm::kFlagCoincident) return fail(MSM_ERR_COINCIDENT, "coincident atoms");
  if (flags & msm::kFlagBadExclusion) return fail(MSM_ERR_INVALID_ARG, "exclusion list entry out of range");
  return MSM_OK;
}

}  // extern "C"
