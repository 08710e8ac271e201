// C ABI of the EnVar library: problem setup (geometry, control map, coarse
// operator inverse), memory layout of the caller-owned state and workspace,
// the time loop with adaptive per-step cycle caps, the anomaly reduction and
// the fixed-ensemble descent loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/envar.h"
#include "common.h"
#include "kernels.h"

namespace envar {

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_OK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(ENVAR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------- problem plan
struct Plan {
  envar_problem p;
  int n;
  int mixed;
  double dt, nu, tol, penalty;
  int cap_max;
  int nlev_grid;        // levels run by the tiled kernels (inv_h > 16)
  int ncoarse;          // levels run by the LDS kernel (top inv_h <= 16 .. 4)
  Geo lev[MAX_LEVELS];  // lev[nlev_grid] is the top of the LDS part
  Tiling mg_tl[3][MAX_LEVELS];  // [8 | 16 | 32 rows][level]
  int mg_tiles[3][MAX_LEVELS];
  Tiling sk_tl[2];              // predictor / projection tiles, 8 | 16 rows
  int sk_tiles[2];
  bool rows16;                  // 16-row step tiles align with the cavity and channel rows
  Tiling st_tl;                 // 64 x 8 cost blocks (also the refinement residual tiles)
  int st_tiles;
  long cplane;  // nx * ny
  int ncells;
  std::vector<int> ctrl_cells;  // dense cell index (i + j nx) of each control cell, row-major
  long m;
  int nc;  // coarsest unknowns
  int norm_slots;
  // state layout
  size_t s_meta, s_u, s_v, s_tu, s_tv, s_phi, s_shu, s_shv, s_cmap, s_ainv, s_aidx, s_total;
  size_t s_code[MAX_LEVELS];  // per-level Poisson diagonal codes (levels 0..nlev_grid)
  // velocity sensors on the cavity lid (vector observation): bilinear stencils per channel
  bool obs_ok = false;
  int obs_fi[OBS_CHANNELS][4], obs_fj[OBS_CHANNELS][4];
  double obs_tx[OBS_CHANNELS], obs_ty[OBS_CHANNELS];
};

// The four sensors x = x_cav + 1/5 .. 4/5 on the cavity lid y = 0 (Sec. 4.1). Each
// component is interpolated bilinearly from its own MAC positions: u faces at
// (i h, y0 + (j + 1/2) h), v faces at ((i + 1/2) h, y0 + j h). Every stencil face must
// be an active face (it is for the cavity geometry).
static void make_sensors(Plan& P) {
  const Geo& g = P.lev[0];
  P.obs_ok = P.p.geometry == ENVAR_CAVITY || P.p.geometry == ENVAR_CAVITY_PAPER;
  if (!P.obs_ok) return;
  const double h = g.h, y0 = -1.0;
  for (int s = 0; s < 4; ++s) {
    const double xs = P.p.x_cav + (s + 1) / 5.0, ys = 0.0;
    for (int comp = 0; comp < 2; ++comp) {
      const int c = 2 * s + comp;
      const double ox = comp == 0 ? 0.0 : 0.5 * h, oy = comp == 0 ? y0 + 0.5 * h : y0;
      const double fx = (xs - ox) / h, fy = (ys - oy) / h;
      const int i = (int)std::floor(fx), j = (int)std::floor(fy);
      P.obs_tx[c] = fx - i;
      P.obs_ty[c] = fy - j;
      const int di[4] = {0, 1, 0, 1}, dj[4] = {0, 0, 1, 1};
      for (int q = 0; q < 4; ++q) {
        const int fi = i + di[q], fj = j + dj[q];
        P.obs_fi[c][q] = fi;
        P.obs_fj[c][q] = fj;
        const bool active = comp == 0 ? (g.fluid(fi - 1, fj) && g.fluid(fi, fj)) : (g.fluid(fi, fj - 1) && g.fluid(fi, fj));
        if (!active) P.obs_ok = false;
      }
    }
  }
}

static Geo make_geo(int n, int geometry, double x_cav) {
  Geo g;
  g.n = n;
  g.nx = 4 * n;
  g.h = 1.0 / n;
  g.slip_top = 0;
  g.slip_i0 = -1;
  g.slip_i1 = 1 << 30;
  g.uconv = 2.0 / 3.0;  // bulk speed of the parabola 4 y (1 - y)
  if (geometry == ENVAR_CAVITY || geometry == ENVAR_CAVITY_PAPER) {
    g.ny = geometry == ENVAR_CAVITY ? 2 * n : n + n / 2;
    g.jc = n;
    g.ic0 = (int)std::lround(x_cav * n);
    g.ic1 = g.ic0 + n;
  } else {
    g.ny = n;
    g.jc = 0;
    g.ic0 = g.ic1 = 0;
  }
  if (geometry == ENVAR_CAVITY_PAPER) {
    // symmetry top; lower wall no-slip for x_cav - 0.4 <= x <= x_cav + 1.75, slip beyond
    g.slip_top = 1;
    g.uconv = 1.0;
    const double xs0 = x_cav - 0.4, xs1 = x_cav + 1.0 + 0.75;
    for (int i = 0; i <= g.nx; ++i) {
      const double x = i * g.h;
      if (x < xs0) g.slip_i0 = i;
      if (x > xs1 && g.slip_i1 > g.nx) g.slip_i1 = i;
    }
  }
  g.pitch = ((g.nx + 1 + 15) / 16) * 16;
  g.rows = g.ny + 1;
  return g;
}

static int make_plan(const envar_problem* pin, Plan& P) {
  if (!pin) return fail(ENVAR_EINVAL, "problem is NULL");
  P.p = *pin;
  envar_problem& p = P.p;
  if (p.inv_h < 16 || p.inv_h % 16 != 0 || p.inv_h > 2048)
    return fail(ENVAR_EINVAL, "inv_h must be a multiple of 16 in [16, 2048], got %d", p.inv_h);
  if (p.geometry != ENVAR_CAVITY && p.geometry != ENVAR_CHANNEL && p.geometry != ENVAR_CAVITY_PAPER)
    return fail(ENVAR_EINVAL, "unknown geometry %d", p.geometry);
  if (p.precision != ENVAR_FP64 && p.precision != ENVAR_MIXED)
    return fail(ENVAR_EINVAL, "unknown precision %d", p.precision);
  if (!(p.Re > 0.0) || !std::isfinite(p.Re)) return fail(ENVAR_EINVAL, "Re must be positive");
  if (p.x_cav <= 0.0) p.x_cav = 1.25;
  if (std::fabs(p.x_cav * 4.0 - std::round(p.x_cav * 4.0)) > 1e-12 || p.x_cav + 1.0 > 4.0)
    return fail(ENVAR_EINVAL, "x_cav must be a multiple of 1/4 with the cavity inside [0, 4]");
  P.n = p.inv_h;
  P.mixed = p.precision == ENVAR_MIXED;
  P.dt = p.dt > 0.0 ? p.dt : 0.064 / p.inv_h;
  P.nu = 1.0 / p.Re;
  P.penalty = p.penalty < 0.0 ? 1e-3 : p.penalty;
  // The solves stop at dt max|r| <= tol on the FP64 residual; the divergence of the projected
  // face velocities is the same quantity computed another way and differs by rounding (about
  // 1e-14 at tol = 1e-10), so the stopping test keeps a 0.1% margin below the requested bound.
  P.tol = (p.div_tol > 0.0 ? p.div_tol : (P.mixed ? 1e-10 : 1e-12)) * (1.0 - 1e-3);
  P.cap_max = p.max_cycles > 0 ? std::min(p.max_cycles, 200) : 30;
  P.norm_slots = P.cap_max + 2;
  // levels
  int nl = 0;
  for (int n = P.n; n > 16; n /= 2) ++nl;
  P.nlev_grid = nl;
  P.lev[0] = make_geo(P.n, p.geometry, p.x_cav);
  for (int l = 1; l <= nl; ++l) P.lev[l] = P.lev[l - 1].coarser();
  const int ntop = P.lev[nl].n;  // 16
  P.ncoarse = 0;
  for (int n = ntop; n >= 4; n /= 2) ++P.ncoarse;
  if (ntop != 16 || P.ncoarse != 3 || P.lev[nl].nx != 64 || P.lev[nl].ny > 32)
    return fail(ENVAR_EINVAL, "internal: the LDS levels must be 16, 8, 4 on a 64 x (<= 32) top box");
  for (int l = 0; l < nl; ++l)
    for (int v = 0; v < 3; ++v) {
      P.mg_tl[v][l] = Tiling::make(P.lev[l], 8 << v, P.mixed ? mg_tw<float>() : mg_tw<double>());
      P.mg_tiles[v][l] = P.mg_tl[v][l].count();
    }
  const Geo& g = P.lev[0];
  P.st_tl = Tiling::make(g, COST_TH);
  P.st_tiles = P.st_tl.count();
  for (int v = 0; v < 2; ++v) {
    P.sk_tl[v] = Tiling::make(g, v ? 16 : 8);
    P.sk_tiles[v] = P.sk_tl[v].count();
  }
  P.rows16 = g.jc % 16 == 0 && (g.ny - g.jc) % 16 == 0;
  P.cplane = (long)g.nx * g.ny;
  P.ncells = 0;
  for (int j = 0; j < g.ny; ++j)
    for (int i = 0; i < g.nx; ++i) P.ncells += g.fluid(i, j);
  // control region, row-major over fluid cells whose centre lies inside
  P.ctrl_cells.clear();
  for (int j = 0; j < g.ny; ++j)
    for (int i = 0; i < g.nx; ++i) {
      if (!g.fluid(i, j)) continue;
      const double x = (i + 0.5) * g.h;
      const double y = (p.geometry == ENVAR_CHANNEL ? 0.0 : -1.0) + (j + 0.5) * g.h;
      bool in = false;
      if (p.region == ENVAR_REGION_COLUMN)
        in = x > p.x_cav && x < p.x_cav + 1.0;
      else if (p.region == ENVAR_REGION_CAVITY)
        in = x > p.x_cav && x < p.x_cav + 1.0 && y < 0.0;
      else if (p.region == ENVAR_REGION_BOX)
        in = x >= p.box[0] && x <= p.box[1] && y >= p.box[2] && y <= p.box[3];
      else
        return fail(ENVAR_EINVAL, "unknown region %d", p.region);
      if (in) P.ctrl_cells.push_back(j * g.nx + i);
    }
  P.m = 2 * (long)P.ctrl_cells.size();
  make_sensors(P);
  // coarsest level
  Geo gc = P.lev[nl];
  for (int l = 1; l < P.ncoarse; ++l) gc = gc.coarser();
  P.nc = 0;
  for (int j = 0; j < gc.ny; ++j)
    for (int i = 0; i < gc.nx; ++i) P.nc += gc.fluid(i, j);
  if (P.nc > MAX_COARSE_UNKNOWNS || P.nc * P.nc > COARSE_INV_MAX)
    return fail(ENVAR_EINVAL, "coarsest level too large (%d unknowns)", P.nc);
  // state layout
  const long pl = g.plane();
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  P.s_meta = take(256);
  P.s_u = take(pl * 8);
  P.s_v = take(pl * 8);
  P.s_tu = take(pl * 8);
  P.s_tv = take(pl * 8);
  P.s_phi = take(pl * 8);
  P.s_shu = take(P.cplane * 8);
  P.s_shv = take(P.cplane * 8);
  P.s_cmap = take(pl * 4);
  P.s_ainv = take((size_t)P.nc * P.nc * 8);
  P.s_aidx = take((size_t)P.nc * 4);
  for (int l = 0; l <= nl; ++l) P.s_code[l] = take((size_t)P.lev[l].plane());
  P.s_total = o;
  return ENVAR_OK;
}

// workspace layout of a forward over nmem members
struct WS {
  size_t u, v, us, vs, us2, vs2, tuA, tvA, tuB, tvB, phiA, phiB, phiC, phiQ, phiR, b0, e0, r0, r1;
  size_t lphiA[MAX_LEVELS], lphiB[MAX_LEVELS], lb[MAX_LEVELS];
  size_t s1u, s1v, s2part, norms, stats, divmax;
  size_t total;
};

// `stride` (optional) receives each buffer's bytes per member: every buffer is member-major, so
// the members [a, b) of a workspace are a workspace of their own at offsets + a * stride.
static WS make_ws(const Plan& P, int nmem, WS* stride = nullptr) {
  WS w{}, st{};
  size_t o = 0;
  auto take = [&](size_t& field, size_t& sfield, size_t per_member) {
    field = o;
    sfield = per_member;
    o = align256(o + (size_t)nmem * per_member);
  };
  const size_t pl = (size_t)P.lev[0].plane();
  const size_t tsz = 8;  // tendency storage (FP64 in both precisions)
  const size_t vsz = P.mixed ? 4 : 8;  // V-cycle storage
  take(w.u, st.u, pl * 8);
  take(w.v, st.v, pl * 8);
  take(w.us, st.us, pl * 8);    // u*, v* of even steps
  take(w.vs, st.vs, pl * 8);
  take(w.us2, st.us2, pl * 8);  // u*, v* of odd steps (the fused predictor reads the other parity)
  take(w.vs2, st.vs2, pl * 8);
  take(w.tuA, st.tuA, pl * tsz);
  take(w.tvA, st.tvA, pl * tsz);
  take(w.tuB, st.tuB, pl * tsz);
  take(w.tvB, st.tvB, pl * tsz);
  take(w.phiA, st.phiA, pl * 8);
  if (!P.mixed) take(w.phiB, st.phiB, pl * 8);
  take(w.phiC, st.phiC, pl * 8);  // previous pressure / next warm start
  take(w.phiQ, st.phiQ, pl * 8);  // pressure two steps back (quadratic warm start)
  // FP64: pressure three steps back (cubic warm start: 2.09 -> 1.78 V-cycles per step at the
  // benchmark shape); mixed precision keeps the quadratic one (1.30 refinement passes per step
  // against 1.46 with the cubic)
  if (!P.mixed) take(w.phiR, st.phiR, pl * 8);
  take(w.b0, st.b0, pl * 8);
  if (P.mixed) {
    take(w.e0, st.e0, pl * 4);
    // the residual carried across the refinement passes of a step (two planes, by pass parity)
    take(w.r0, st.r0, pl * 4);
    take(w.r1, st.r1, pl * 4);
  }
  for (int l = 1; l <= P.nlev_grid; ++l) {
    const size_t lp = (size_t)P.lev[l].plane();
    take(w.lphiA[l], st.lphiA[l], lp * vsz);
    if (l < P.nlev_grid) take(w.lphiB[l], st.lphiB[l], lp * vsz);
    take(w.lb[l], st.lb[l], lp * vsz);
  }
  take(w.s1u, st.s1u, (size_t)P.cplane * 8);
  take(w.s1v, st.s1v, (size_t)P.cplane * 8);
  take(w.s2part, st.s2part, (size_t)P.st_tiles * 8);
  take(w.norms, st.norms, (size_t)P.norm_slots * 8);
  take(w.stats, st.stats, (size_t)STATS_STRIDE * 8);
  take(w.divmax, st.divmax, 8);
  w.total = o;
  if (stride) *stride = st;
  return w;
}

// the workspace of members [a, a + k) of `w`: every buffer offset moved by a members
static WS slice_ws(const WS& w, const WS& stride, int a) {
  static_assert(sizeof(WS) % sizeof(size_t) == 0, "WS holds offsets only");
  WS out = w;
  size_t* d = (size_t*)&out;
  const size_t* sd = (const size_t*)&stride;
  constexpr size_t nf = sizeof(WS) / sizeof(size_t) - 1;  // every field but `total` (the last)
  for (size_t f = 0; f < nf; ++f) d[f] += (size_t)a * sd[f];
  return out;
}

// dense inverse of the coarsest operator (Gauss-Jordan with partial pivoting)
static void coarse_inverse(const Geo& g, std::vector<double>& inv, std::vector<int>& idx) {
  idx.clear();
  std::vector<int> id(g.nx * g.ny, -1);
  for (int j = 0; j < g.ny; ++j)
    for (int i = 0; i < g.nx; ++i)
      if (g.fluid(i, j)) {
        id[j * g.nx + i] = (int)idx.size();
        idx.push_back(j * g.nx + i);
      }
  const int nc = (int)idx.size();
  std::vector<double> A((size_t)nc * nc, 0.0);
  const double ih2 = 1.0 / (g.h * g.h);
  for (int q = 0; q < nc; ++q) {
    const int i = idx[q] % g.nx, j = idx[q] / g.nx;
    A[(size_t)q * nc + q] = -(double)g.diag_count(i, j) * ih2;
    const int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
    for (auto& c : nb)
      if (g.fluid(c[0], c[1])) A[(size_t)q * nc + id[c[1] * g.nx + c[0]]] = ih2;
  }
  inv.assign((size_t)nc * nc, 0.0);
  for (int q = 0; q < nc; ++q) inv[(size_t)q * nc + q] = 1.0;
  for (int c = 0; c < nc; ++c) {
    int pr = c;
    for (int r = c + 1; r < nc; ++r)
      if (std::fabs(A[(size_t)r * nc + c]) > std::fabs(A[(size_t)pr * nc + c])) pr = r;
    if (pr != c)
      for (int k = 0; k < nc; ++k) {
        std::swap(A[(size_t)pr * nc + k], A[(size_t)c * nc + k]);
        std::swap(inv[(size_t)pr * nc + k], inv[(size_t)c * nc + k]);
      }
    const double d = 1.0 / A[(size_t)c * nc + c];
    for (int k = 0; k < nc; ++k) {
      A[(size_t)c * nc + k] *= d;
      inv[(size_t)c * nc + k] *= d;
    }
    for (int r = 0; r < nc; ++r) {
      if (r == c) continue;
      const double f = A[(size_t)r * nc + c];
      if (f == 0.0) continue;
      for (int k = 0; k < nc; ++k) {
        A[(size_t)r * nc + k] -= f * A[(size_t)c * nc + k];
        inv[(size_t)r * nc + k] -= f * inv[(size_t)c * nc + k];
      }
    }
  }
}

template <typename T>
static T* at(void* base, size_t off) {
  return (T*)((char*)base + off);
}
template <typename T>
static const T* at(const void* base, size_t off) {
  return (const T*)((const char*)base + off);
}


// HIP-event sampling of the main kernels on the call's stream
enum { TM_PRED = 0, TM_PRE = 1, TM_POST = 2, TM_RESID = 3, TM_PROJ = 4, TM_CYCLE = 5, TM_N = 6 };
struct Timer {
  bool on = false;
  int every = 1, max_samples = 256;
  std::vector<hipEvent_t> ev;  // [sample][TM_N][2]
  std::vector<unsigned char> rec;  // [sample][TM_N] both edges recorded
  int samples = 0;
  int members = 0;  // members of the timed launches (the first lane's)
  int cur = -1;  // sample index of the current step, -1 = not sampled
  int begin_step(int s, int steps) {
    cur = -1;
    if (!on || s == 0) return 0;
    if ((s - 1) % every != 0 || samples >= max_samples) return 0;
    cur = samples++;
    const size_t need = (size_t)samples * TM_N * 2;
    while (ev.size() < need) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      ev.push_back(e);
    }
    rec.resize((size_t)samples * TM_N, 0);
    return 0;
  }
  void mark(int what, int edge, hipStream_t s) {
    if (cur < 0) return;
    if (hipEventRecord(ev[((size_t)cur * TM_N + what) * 2 + edge], s) == hipSuccess)
      rec[(size_t)cur * TM_N + what] |= (unsigned char)(1 << edge);
  }
  bool recorded(int q, int what) const { return rec[(size_t)q * TM_N + what] == 3; }
  ~Timer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// ---------------------------------------------------------------------------- jobs and merged launches
// A job is one ensemble: a problem, its base state, its workspace and its
// control rows. A batch advances several jobs by one time step each with one
// launch per phase (predictor, every multigrid level, coarse solve,
// refinement residual, projection, bookkeeping): each launch carries one
// segment per job, and jobs may differ in grid, Reynolds number, member count,
// horizon and multigrid depth. A single forward is a batch of one job.
struct Job {
  Plan P;
  WS w;
  void* ws = nullptr;
  const void* state = nullptr;
  const double* ctrl = nullptr;
  int nmem = 0;
  int horizon = 0;
  int step = 0;            // steps launched so far
  bool cold_first = true;  // the state's cold-start flag applies to step 0
  int last_cur = 0;        // pressure buffer of the last solved step
  // sensor series of the vector observation: obs[nmem][OBS_CHANNELS][obs_K], a sample every obs_every steps
  double* obs = nullptr;
  int obs_K = 0, obs_every = 1;
  // tile heights (8 | 16) of the predictor, the projection and each tiled multigrid level
  int rows_pred = 8, rows_proj = 8;
  int rows_mg[MAX_LEVELS] = {16, 16, 16, 16, 16, 16, 16, 16, 16, 16, 16, 16};
  template <typename T>
  T* w_(size_t off) const {
    return at<T>(ws, off);
  }
  double* phi(int k) const { return w_<double>(k ? w.phiC : w.phiA); }
  // the residual carried after refinement pass k (pass k reads plane k - 1, writes plane k)
  float* rplane(int k) const { return w_<float>((k & 1) ? w.r1 : w.r0); }
  double* ustar(int p) const { return w_<double>(p ? w.us2 : w.us); }
  double* vstar(int p) const { return w_<double>(p ? w.vs2 : w.vs); }
};

template <typename A>
static void seg_add(Multi<A>& m, const A& a, int wgs) {
  m.seg[m.nseg] = a;
  m.start[m.nseg + 1] = m.start[m.nseg] + wgs;
  ++m.nseg;
}
template <typename A>
static Multi<A> seg_begin() {
  Multi<A> m;
  std::memset((void*)&m, 0, sizeof m);
  return m;
}

// ---------------------------------------------------------------------------- launch arguments
// Builders shared by the time step and the tile tuner. `rows` is the tile
// height (8 or 16) of the launch; k is the V-cycle pass.
static int vidx(int rows) { return rows == 16 ? 1 : 0; }
static int mg_vidx(int rows) { return rows == 32 ? 2 : rows == 16 ? 1 : 0; }

static PredArgs<double> pred_args(const Job& j, int rows, bool fused) {
  const Plan& P = j.P;
  const WS& w = j.w;
  const bool even = (j.step & 1) == 0;
  const int par = j.step & 1;
  PredArgs<double> a{};
  a.g = P.lev[0];
  a.tiling = P.sk_tl[vidx(rows)];
  a.trows = rows;
  a.ntiles = P.sk_tiles[vidx(rows)];
  a.nmem = j.nmem;
  a.plane = P.lev[0].plane();
  a.nu = P.nu;
  a.dt = P.dt;
  a.cold_flag = (j.step == 0 && j.cold_first) ? at<int>(j.state, P.s_meta) : nullptr;
  a.us = j.ustar(par);
  a.vs = j.vstar(par);
  if (fused) {  // projection of the previous step: its u*, v* and phi (the other parity)
    a.fused = 1;
    a.u = j.ustar(par ^ 1);
    a.v = j.vstar(par ^ 1);
    a.phi = j.phi(par ^ 1);
    a.phi_next = j.phi(par);
    a.phi_old = j.w_<double>(w.phiQ);
    a.phi_old2 = P.mixed ? nullptr : j.w_<double>(w.phiR);
    a.stats = j.w_<double>(w.stats);
    a.shu = at<double>(j.state, P.s_shu);
    a.shv = at<double>(j.state, P.s_shv);
    a.s1u = j.w_<double>(w.s1u);
    a.s1v = j.w_<double>(w.s1v);
    a.s2part = j.w_<double>(w.s2part);
    a.divmax = j.w_<double>(w.divmax);
    a.cost_tiling = P.st_tl;
    a.cost_ntiles = P.st_tiles;
    a.cplane = P.cplane;
  } else {
    a.u = j.w_<double>(w.u);
    a.v = j.w_<double>(w.v);
  }
  a.tu_prev = j.w_<double>(even ? w.tuA : w.tuB);
  a.tv_prev = j.w_<double>(even ? w.tvA : w.tvB);
  a.tu = j.w_<double>(even ? w.tuB : w.tuA);
  a.tv = j.w_<double>(even ? w.tvB : w.tvA);
  a.b = j.w_<double>(w.b0);
  a.ctrl = j.ctrl;
  a.m = P.m;
  a.nctrl = (int)(P.m / 2);
  a.cmap = at<int>(j.state, P.s_cmap);
  a.norms = j.w_<double>(w.norms);
  a.norm_slots = P.norm_slots;
  return a;
}

// the projection that closes a forward (cur: parity of its last step)
static ProjArgs proj_args(const Job& j, int rows, int cur) {
  const Plan& P = j.P;
  const WS& w = j.w;
  ProjArgs pj{};
  pj.g = P.lev[0];
  pj.tiling = P.sk_tl[vidx(rows)];
  pj.trows = rows;
  pj.ntiles = P.sk_tiles[vidx(rows)];
  pj.cost_tiling = P.st_tl;
  pj.cost_ntiles = P.st_tiles;
  pj.nmem = j.nmem;
  pj.plane = P.lev[0].plane();
  pj.cplane = P.cplane;
  pj.dt = P.dt;
  pj.u = j.w_<double>(w.u);
  pj.v = j.w_<double>(w.v);
  pj.us = j.ustar(cur);
  pj.vs = j.vstar(cur);
  pj.phi = j.phi(cur);
  pj.phi_next = j.phi(cur ^ 1);
  pj.phi_old = j.w_<double>(w.phiQ);
  pj.phi_old2 = P.mixed ? nullptr : j.w_<double>(w.phiR);
  pj.stats = j.w_<double>(w.stats);
  pj.shu = at<double>(j.state, P.s_shu);
  pj.shv = at<double>(j.state, P.s_shv);
  pj.s1u = j.w_<double>(w.s1u);
  pj.s1v = j.w_<double>(w.s1v);
  pj.s2part = j.w_<double>(w.s2part);
  pj.divmax = j.w_<double>(w.divmax);
  return pj;
}

template <typename T>
static MGArgs<T> level_args(const Job& j, int l, int k, int rows) {
  const Plan& P = j.P;
  MGArgs<T> a{};
  a.g = P.lev[l];
  a.gc = P.lev[l + 1];
  a.tiling = P.mg_tl[mg_vidx(rows)][l];
  a.trows = rows;
  a.ntiles = P.mg_tiles[mg_vidx(rows)][l];
  a.nmem = j.nmem;
  a.plane = P.lev[l].plane();
  a.cplane_c = P.lev[l + 1].plane();
  a.norms = j.w_<double>(j.w.norms);
  a.norm_slots = P.norm_slots;
  a.tol = P.tol;
  a.dt = P.dt;
  a.code = at<unsigned char>(j.state, P.s_code[l]);
  a.codec = at<unsigned char>(j.state, P.s_code[l + 1]);
  a.k = k;
  return a;
}

template <typename T>
static MGArgs<T> pre_args(const Job& j, int l, int k, int rows) {
  const WS& w = j.w;
  const bool mixed = j.P.mixed;
  MGArgs<T> a = level_args<T>(j, l, k, rows);
  if (l == 0) {
    const int cur = j.step & 1;
    a.phi_in = mixed ? nullptr : (const T*)j.phi(cur);
    a.b = mixed ? nullptr : (const T*)j.w_<double>(w.b0);
    a.zero_guess = mixed ? 1 : 0;
    a.phi_out = mixed ? (T*)j.w_<float>(w.e0) : (T*)j.w_<double>(w.phiB);
    if (mixed && k <= 1) {  // first pass: the residual of the warm-started FP64 pressure is formed here
      a.pre_mode = PRE_FIRST;
      a.phi64 = j.phi(cur);
      a.b64 = j.w_<double>(w.b0);
      a.r_out = (T*)j.rplane(0);
      a.rslot = 0;
    } else if (mixed) {
      // later passes: the residual carried from the previous pass's post kernel, re-formed from the
      // FP64 pressure into the same plane while its norm exceeds 1e3 x the tolerance (so that the
      // rounding of a large carried residual, relative 6e-8, never reaches the tolerance)
      a.pre_mode = PRE_LATER;
      a.b = (const T*)j.rplane(k - 1);
      a.r_out = (T*)j.rplane(k - 1);
      a.phi64 = j.phi(cur);
      a.b64 = j.w_<double>(w.b0);
      a.anchor = 1e3 * j.P.tol;
    }
  } else {
    a.phi_in = nullptr;
    a.b = j.w_<T>(w.lb[l]);
    a.zero_guess = 1;
    a.phi_out = j.w_<T>(w.lphiB[l]);
  }
  a.bc = j.w_<T>(w.lb[l + 1]);
  return a;
}

template <typename T>
static MGArgs<T> post_args(const Job& j, int l, int k, int rows) {
  const WS& w = j.w;
  const bool mixed = j.P.mixed;
  MGArgs<T> a = level_args<T>(j, l, k, rows);
  a.phic = j.w_<T>(w.lphiA[l + 1]);
  if (l == 0) {
    const int cur = j.step & 1;
    a.phi_in = mixed ? (const T*)j.w_<float>(w.e0) : (const T*)j.w_<double>(w.phiB);
    a.b = mixed ? (const T*)j.rplane(k - 1) : (const T*)j.w_<double>(w.b0);
    a.phi_out = mixed ? nullptr : (T*)j.phi(cur);
    a.add_to = mixed ? j.phi(cur) : nullptr;
    if (mixed) a.r_out = (T*)j.rplane(k);  // phi64 += e, r - L e into plane k; a skipped member carries its norm
    a.write_norm = 1;
  } else {
    a.phi_in = j.w_<T>(w.lphiB[l]);
    a.b = j.w_<T>(w.lb[l]);
    a.phi_out = j.w_<T>(w.lphiA[l]);
  }
  return a;
}

template <typename T>
static CoarseArgs coarse_args(const Job& j, int k) {
  const Plan& P = j.P;
  const WS& w = j.w;
  const int L = P.nlev_grid;
  CoarseArgs c{};
  c.g = P.lev[L];
  c.nlev = P.ncoarse;
  c.nmem = j.nmem;
  c.plane = P.lev[L].plane();
  c.ainv = at<double>(j.state, P.s_ainv);
  c.aidx = at<int>(j.state, P.s_aidx);
  c.nc = P.nc;
  c.norms = j.w_<double>(w.norms);
  c.norm_slots = P.norm_slots;
  c.k = k;
  c.tol = P.tol;
  c.dt = P.dt;
  c.nsweep_pre = P.mixed ? mg_ns<float>() : mg_ns<double>();
  c.nsweep_post = c.nsweep_pre;
  if (L == 0) {  // the whole V-cycle runs in LDS
    const int cur = j.step & 1;
    if (P.mixed) {
      c.phi = j.w_<float>(w.e0);
      c.b = j.w_<float>(w.r0);
      c.add_to = j.phi(cur);
    } else {
      c.phi = j.phi(cur);
      c.b = j.w_<double>(w.b0);
      c.warm = 1;
      c.write_norm = 1;
    }
  } else {
    c.phi = j.w_<T>(w.lphiA[L]);
    c.b = j.w_<T>(w.lb[L]);
  }
  return c;
}

static ResidArgs resid_args(const Job& j, int k) {
  const Plan& P = j.P;
  ResidArgs r{};
  r.g = P.lev[0];
  r.tiling = P.st_tl;
  r.ntiles = P.st_tiles;
  r.nmem = j.nmem;
  r.plane = P.lev[0].plane();
  r.phi = j.phi(j.step & 1);
  r.b = j.w_<double>(j.w.b0);
  r.r = j.w_<float>(j.w.r0);
  r.norms = j.w_<double>(j.w.norms);
  r.norm_slots = P.norm_slots;
  r.tol = P.tol;
  r.dt = P.dt;
  r.k = k;
  return r;
}

// One launch per tile height present among the jobs (the kernels take the
// height as a compile-time parameter); `rows_of` gives a job's height for the
// phase, or 0 when the job has no work in it.
template <typename A, typename RowsOf, typename Make, typename Launch>
static void grouped(const std::vector<Job*>& J, RowsOf rows_of, Make make, Launch launch) {
  for (int rows : {8, 16, 32}) {
    auto m = seg_begin<A>();
    for (Job* j : J)
      if (rows_of(*j) == rows) {
        const A a = make(*j, rows);
        seg_add(m, a, a.ntiles * a.nmem);
      }
    if (m.nseg) launch(m);
  }
}

// A job runs at most its own max_cycles passes whatever the batch's cap (its norm slots are
// sized by it).
static int job_cap(const Job& j, int cap) { return std::min(cap, j.P.cap_max); }

// A job whose passes beyond the step's cap can run in the tail kernel (one workgroup per member).
static bool tail_fits(const Job& j) { return j.P.nlev_grid >= 1 && j.P.nlev_grid <= TAIL_MAX_LEV; }

template <typename T>
static TailArgs<T> tail_args(const Job& j, int k0, int k1) {
  TailArgs<T> t{};
  t.nlev = j.P.nlev_grid;
  t.k0 = k0;
  t.k1 = k1;
  t.mixed = j.P.mixed;
  for (int l = 0; l < t.nlev; ++l) {
    t.pre[l] = pre_args<T>(j, l, k0, TAIL_ROWS);
    t.post[l] = post_args<T>(j, l, k0, TAIL_ROWS);
  }
  t.coarse = coarse_args<T>(j, k0);
  if (j.P.mixed) {
    t.rpl[0] = (T*)j.rplane(0);
    t.rpl[1] = (T*)j.rplane(1);
  }
  return t;
}

// the step record of a job's members (the tail fills every norm slot up to max_cycles)
static BookArgs book_args(const Job& j, int cap, bool tail) {
  BookArgs bk{};
  bk.nmem = j.nmem;
  bk.norm_slots = j.P.norm_slots;
  bk.cap = tail ? j.P.cap_max : job_cap(j, cap);
  bk.slot_base = j.P.mixed ? 1 : 0;
  bk.tol = j.P.tol;
  bk.norms = j.w_<double>(j.w.norms);
  bk.stats = j.w_<double>(j.w.stats);
  return bk;
}

// Returns whether the tail launches wrote every job's step record (then no bookkeeping launch is
// needed): when every job has a tail launch this step and `book` is set.
template <typename TT>
static bool batch_pressure(const std::vector<Job*>& J, hipStream_t st, int cap, bool tail, bool book, Timer* tm) {
  typedef TT T;  // V-cycle type
  const bool mixed = J[0]->P.mixed;
  const int k_timed = mixed ? 1 : 0;
  // jobs that run pass k (FP64: k = 0 .. cap-1; mixed: k = 1 .. cap)
  auto in_pass = [&](int k) {
    std::vector<Job*> Jk;
    for (Job* j : J)
      if (mixed ? k <= job_cap(*j, cap) : k < job_cap(*j, cap)) Jk.push_back(j);
    return Jk;
  };
  auto vcycle = [&](int k, const std::vector<Job*>& Jk) {
    int Lmax = 0;
    for (Job* j : Jk) Lmax = std::max(Lmax, j->P.nlev_grid);
    const bool timed = tm && k == k_timed;
    if (timed) tm->mark(TM_CYCLE, 0, st);
    for (int l = 0; l < Lmax; ++l) {
      if (timed && l == 0) tm->mark(TM_PRE, 0, st);
      grouped<MGArgs<T>>(
          Jk, [&](const Job& j) { return l < j.P.nlev_grid ? j.rows_mg[l] : 0; },
          [&](const Job& j, int rows) { return pre_args<T>(j, l, k, rows); },
          [&](const Multi<MGArgs<T>>& m) { launch_mg_pre<T>(m, st); });
      if (timed && l == 0) tm->mark(TM_PRE, 1, st);
    }
    {
      auto m = seg_begin<CoarseArgs>();
      for (Job* j : Jk) seg_add(m, coarse_args<T>(*j, k), j->nmem);
      launch_mg_coarse<T>(m, st);
    }
    for (int l = Lmax - 1; l >= 0; --l) {
      if (timed && l == 0) tm->mark(TM_POST, 0, st);
      grouped<MGArgs<T>>(
          Jk, [&](const Job& j) { return l < j.P.nlev_grid ? j.rows_mg[l] : 0; },
          [&](const Job& j, int rows) { return post_args<T>(j, l, k, rows); },
          [&](const Multi<MGArgs<T>>& m) {
            launch_mg_post<T>(m, l > 0 ? POST_PLAIN : mixed ? POST_REFINE : POST_NORM, st);
          });
      if (timed && l == 0) tm->mark(TM_POST, 1, st);
    }
    if (timed && !mixed) tm->mark(TM_CYCLE, 1, st);
  };
  // standalone FP64 residual into slot k (k < 0: each job's last slot, its own cap): for every
  // job when `all`, else only for jobs whose finest level runs in the one-workgroup coarse
  // kernel (the tiled finest pre kernel forms it otherwise)
  auto resid = [&](int k, const std::vector<Job*>& Jk, bool all) {
    auto m = seg_begin<ResidArgs>();
    for (Job* j : Jk) {
      if (!all && j->P.nlev_grid > 0) continue;
      const ResidArgs r = resid_args(*j, k < 0 ? job_cap(*j, cap) : k);
      seg_add(m, r, r.ntiles * r.nmem);
    }
    if (m.nseg > 0) launch_resid64(m, st);
  };
  if (!mixed) {
    for (int k = 0; k < cap; ++k) {
      const std::vector<Job*> Jk = in_pass(k);
      if (!Jk.empty()) vcycle(k, Jk);
    }
  } else {
    // slot 0 holds the initial residual (the first pass's finest pre kernel), slot k the residual
    // after pass k (that pass's finest post kernel; for jobs without a tiled level, the standalone
    // residual launches)
    resid(0, J, false);
    for (int k = 1; k <= cap; ++k) {
      const std::vector<Job*> Jk = in_pass(k);
      if (Jk.empty()) break;
      vcycle(k, Jk);
      resid(k, in_pass(k + 1), false);
      if (tm && k == k_timed) tm->mark(TM_CYCLE, 1, st);
    }
    // the last pass's residual: tiled jobs carry it out of their finest post kernel; jobs whose
    // finest level runs in the coarse kernel form it here
    if (tm) tm->mark(TM_RESID, 0, st);
    resid(-1, J, false);
    if (tm) tm->mark(TM_RESID, 1, st);
  }
  // the passes beyond the cap, up to each job's own max_cycles, for the members that need them
  // (mixed: passes cap + 1 .. max_cycles; FP64: V-cycles cap .. max_cycles - 1)
  if (!tail) return false;
  bool booked = book;
  for (Job* j : J) {
    const int c = job_cap(*j, cap);
    booked = booked && (mixed ? c + 1 : c) <= (mixed ? j->P.cap_max : j->P.cap_max - 1);
  }
  for (Job* j : J) {
    const int c = job_cap(*j, cap);
    const int k0 = mixed ? c + 1 : c, k1 = mixed ? j->P.cap_max : j->P.cap_max - 1;
    if (k0 > k1) continue;
    TailArgs<T> ta = tail_args<T>(*j, k0, k1);
    if (booked) {
      ta.book = book_args(*j, cap, true);
      ta.book_member = 1;
    }
    launch_mg_tail<T>(ta, j->nmem, st);
  }
  return booked;
}

// One time step of every job of the batch (each at its own step index).
template <typename TT>
static int batch_step(const std::vector<Job*>& J, hipStream_t st, int cap, bool tail, Timer* tm) {
  // the first step of a job starts from u^n; later steps fuse the previous step's projection
  if (tm) tm->mark(TM_PRED, 0, st);
  for (const bool fused : {false, true})
    grouped<PredArgs<double>>(
        J, [&](const Job& j) { return (j.step > 0) == fused ? j.rows_pred : 0; },
        [&](const Job& j, int rows) { return pred_args(j, rows, fused); },
        [&](const Multi<PredArgs<double>>& m) { launch_predictor<double>(m, st); });
  if (tm) tm->mark(TM_PRED, 1, st);
  // sensors read the step counter that the record advances, so a batch with sensors keeps the
  // bookkeeping launch after them
  bool any_obs = false;
  for (const Job* j : J) any_obs = any_obs || j->obs != nullptr;
  const bool booked = batch_pressure<TT>(J, st, cap, tail, !any_obs, tm);
  {
    auto m = seg_begin<SensorArgs>();
    for (Job* j : J) {
      if (!j->obs) continue;
      const Plan& P = j->P;
      const int par = j->step & 1;
      SensorArgs a{};
      a.g = P.lev[0];
      a.nmem = j->nmem;
      a.plane = P.lev[0].plane();
      a.dt = P.dt;
      a.us = j->ustar(par);
      a.vs = j->vstar(par);
      a.phi = j->phi(par);
      a.stats = j->w_<double>(j->w.stats);
      a.obs = j->obs;
      a.K = j->obs_K;
      a.every = j->obs_every;
      std::memcpy(a.fi, P.obs_fi, sizeof a.fi);
      std::memcpy(a.fj, P.obs_fj, sizeof a.fj);
      std::memcpy(a.tx, P.obs_tx, sizeof a.tx);
      std::memcpy(a.ty, P.obs_ty, sizeof a.ty);
      seg_add(m, a, (j->nmem * OBS_CHANNELS + 63) / 64);
    }
    if (m.nseg) launch_sensors(m, st);
  }
  if (!booked) {
    auto m = seg_begin<BookArgs>();
    for (Job* j : J) {
      const BookArgs bk = book_args(*j, cap, tail);
      seg_add(m, bk, (j->nmem + 63) / 64);
    }
    launch_step_book(m, st);
  }
  HIP_OK(hipGetLastError());
  return ENVAR_OK;
}

template <typename TT>
static void init_members(const Job& j, hipStream_t s) {
  const Plan& P = j.P;
  const WS& w = j.w;
  InitArgs<double> ia{};
  ia.nmem = j.nmem;
  ia.ntiles = P.st_tiles;
  ia.plane = P.lev[0].plane();
  ia.cplane = P.cplane;
  ia.bu = at<double>(j.state, P.s_u);
  ia.bv = at<double>(j.state, P.s_v);
  ia.btu = at<double>(j.state, P.s_tu);
  ia.btv = at<double>(j.state, P.s_tv);
  ia.bphi = at<double>(j.state, P.s_phi);
  ia.u = j.w_<double>(w.u);
  ia.v = j.w_<double>(w.v);
  ia.us = j.w_<double>(w.us);
  ia.vs = j.w_<double>(w.vs);
  ia.us2 = j.w_<double>(w.us2);
  ia.vs2 = j.w_<double>(w.vs2);
  ia.phi = j.w_<double>(w.phiA);
  ia.phi2 = j.w_<double>(w.phiC);
  ia.tu = j.w_<double>(w.tuA);
  ia.tv = j.w_<double>(w.tvA);
  ia.s1u = j.w_<double>(w.s1u);
  ia.s1v = j.w_<double>(w.s1v);
  ia.s2part = j.w_<double>(w.s2part);
  ia.stats = j.w_<double>(w.stats);
  ia.divmax = j.w_<double>(w.divmax);
  launch_init_members<double>(ia, s);
}

// J of a finished job (and optionally its fields / the spin-up store)
static void finish_job(const Job& j, double* J_dev, double* fields_dev, bool spinup_store, hipStream_t s) {
  const Plan& P = j.P;
  const WS& w = j.w;
  {
    // the projection of the last step (earlier ones ran fused into the next predictor)
    auto m = seg_begin<ProjArgs>();
    const ProjArgs pj = proj_args(j, j.rows_proj, j.last_cur);
    seg_add(m, pj, pj.ntiles * pj.nmem);
    launch_project_cost(m, s);
  }
  if (J_dev) {
    FinalArgs fa{};
    fa.g = P.lev[0];
    fa.nmem = j.nmem;
    fa.ntiles = P.st_tiles;
    fa.cplane = P.cplane;
    fa.K = j.horizon;
    fa.dt = P.dt;
    fa.penalty = P.penalty;
    fa.s1u = j.w_<double>(w.s1u);
    fa.s1v = j.w_<double>(w.s1v);
    fa.s2part = j.w_<double>(w.s2part);
    fa.ctrl = j.ctrl;
    fa.m = P.m;
    fa.J = J_dev;
    fa.stats = j.w_<double>(w.stats);
    launch_finalize_J(fa, s);
  }
  if (fields_dev)
    launch_fields_out(P.lev[0], P.lev[0].plane(), j.nmem, j.w_<double>(w.u), j.w_<double>(w.v), fields_dev, s);
  if (spinup_store) {
    // the last step wrote its tendency into buffer B when the horizon is odd
    const bool inB = (j.horizon % 2) == 1;
    void* S = (void*)j.state;
    const long pl = P.lev[0].plane();
    double* phi_last = j.phi(j.last_cur);
    launch_store_base<double>(pl, j.w_<double>(w.u), j.w_<double>(w.v), j.w_<double>(inB ? w.tuB : w.tuA),
                              j.w_<double>(inB ? w.tvB : w.tvA), phi_last, at<double>(S, P.s_u), at<double>(S, P.s_v),
                              at<double>(S, P.s_tu), at<double>(S, P.s_tv), at<double>(S, P.s_phi), s);
    launch_clear_flag(at<int>(S, P.s_meta), s);
    launch_shift(P.lev[0], at<double>(S, P.s_u), at<double>(S, P.s_v), at<double>(S, P.s_shu), at<double>(S, P.s_shv),
                 s);
  }
}

// Graph executables, their graphs and capture streams may still have launches
// queued on the stream that replays them when they are retired (a re-key of the
// cycle cap or of the job set, or the end of a call that returns before its
// stream drains). They are kept here with an event recorded on that stream
// after their last launch and destroyed once it has completed.
struct Retired {
  hipEvent_t ev = nullptr;
  hipGraphExec_t x = nullptr;
  hipGraph_t g = nullptr;
  hipStream_t cs = nullptr;
};
static std::mutex g_retired_mu;
static std::vector<Retired> g_retired;

static void destroy_retired(const Retired& r) {
  if (r.x) (void)hipGraphExecDestroy(r.x);
  if (r.g) (void)hipGraphDestroy(r.g);
  if (r.cs) (void)hipStreamDestroy(r.cs);
  if (r.ev) (void)hipEventDestroy(r.ev);
}

// destroy every retired object whose launches have completed
static void reap_retired() {
  std::vector<Retired> done;
  {
    std::lock_guard<std::mutex> lk(g_retired_mu);
    for (size_t k = 0; k < g_retired.size();) {
      const hipError_t q = hipEventQuery(g_retired[k].ev);
      if (q == hipErrorNotReady) {
        ++k;
        continue;
      }
      done.push_back(g_retired[k]);  // completed (or the event failed: nothing left to wait for)
      g_retired[k] = g_retired.back();
      g_retired.pop_back();
    }
  }
  for (const Retired& r : done) destroy_retired(r);
  (void)hipGetLastError();
}

// retire objects whose last launch was queued on `s`
static void retire(Retired r, hipStream_t s) {
  if (!r.x && !r.g && !r.cs) return;
  if (hipEventCreateWithFlags(&r.ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(r.ev, s) != hipSuccess) {
    // no event: wait for the stream instead, then destroy at once
    if (r.ev) (void)hipEventDestroy(r.ev);
    r.ev = nullptr;
    (void)hipStreamSynchronize(s);
    destroy_retired(r);
    (void)hipGetLastError();
    return;
  }
  {
    std::lock_guard<std::mutex> lk(g_retired_mu);
    g_retired.push_back(r);
  }
  reap_retired();
}

// Captured batch steps. All jobs advance together, so a step's launch
// sequence depends on the job set, the step parities and the cycle cap: two
// graphs (one per parity) are kept per (job set, cap) and replayed on `ls`.
struct StepGraphs {
  hipStream_t cs = nullptr;  // capture stream
  hipStream_t ls = nullptr;  // stream the executables are launched on
  hipGraph_t g[2] = {nullptr, nullptr};
  hipGraphExec_t x[2] = {nullptr, nullptr};
  long key[2] = {-1, -1};
  void drop(int p) {
    Retired r;
    r.x = x[p];
    r.g = g[p];
    retire(r, ls);
    x[p] = nullptr;
    g[p] = nullptr;
    key[p] = -1;
  }
  // destroy everything now: the caller has synchronised the launch stream
  void destroy_drained() {
    for (int p = 0; p < 2; ++p) {
      Retired r;
      r.x = x[p];
      r.g = g[p];
      destroy_retired(r);
      x[p] = nullptr;
      g[p] = nullptr;
      key[p] = -1;
    }
    Retired r;
    r.cs = cs;
    destroy_retired(r);
    cs = nullptr;
  }
  ~StepGraphs() {
    drop(0);
    drop(1);
    Retired r;
    r.cs = cs;
    retire(r, ls);
  }
};

// Batch driver shared by envar_forward, envar_forward_batch and the server.
struct Driver {
  int cap = 0;
  int cap_max = 0;
  bool tail = false;         // passes beyond the cap run in the per-member tail kernel
  bool short_graph = false;  // cap pinned to one pass (the tail runs the rest)
  long epoch = 0;  // bumps whenever the job set changes
  StepGraphs G;
  hipEvent_t ev = nullptr;
  bool pending = false;
  std::vector<double> host;  // per-job stats snapshots for the cap monitor
  std::vector<Job*> watched;
  double* pinned = nullptr;
  size_t pinned_n = 0;
  double unconv_seen = 0.0;  // member-steps cut by the cap, summed over the watched jobs at the last poll
  Driver() { reap_retired(); }
  ~Driver() {
    drain();  // no copy into the pinned buffer may outlive it
    if (ev) (void)hipEventDestroy(ev);
    if (pinned) (void)hipHostFree(pinned);
  }
  int ensure_pinned(size_t n) {
    if (n <= pinned_n) return ENVAR_OK;
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    pinned_n = 0;
    HIP_OK(hipHostMalloc((void**)&pinned, n * sizeof(double), hipHostMallocDefault));
    pinned_n = n;
    return ENVAR_OK;
  }
  int absorb_now(const std::vector<Job*>& J, hipStream_t s) {
    // a poll started before the job set changed would later be absorbed over the old job count
    // (dropping the new jobs from the cap) and may still be copying into the buffer that is
    // resized below: wait for it and let this synchronous snapshot supersede it
    drain();
    size_t n = 0;
    for (Job* j : J) n += (size_t)j->nmem * STATS_STRIDE;
    int rc = ensure_pinned(n);
    if (rc) return rc;
    size_t o = 0;
    for (Job* j : J) {
      HIP_OK(hipMemcpyAsync(pinned + o, j->w_<double>(j->w.stats), (size_t)j->nmem * STATS_STRIDE * 8,
                            hipMemcpyDeviceToHost, s));
      o += (size_t)j->nmem * STATS_STRIDE;
    }
    HIP_OK(hipStreamSynchronize(s));
    absorb(n);
    return ENVAR_OK;
  }
  void absorb(size_t n) {
    int mx = 0;
    double unconv = 0.0;
    for (size_t q = 0; q < n; q += STATS_STRIDE) {
      mx = std::max(mx, (int)std::ceil(pinned[q + ST_RECENT]));
      unconv += pinned[q + ST_UNCONV];
    }
    // ST_RECENT decays by one cycle per 16 steps: the cap follows what the members needed
    // lately (start-up transients fade). With the tail kernel the passes beyond the cap still
    // run, per member, up to its max_cycles, so the cap only decides which passes are level
    // launches; without it the cap keeps one cycle of headroom above the recent need. A member
    // that converges within its passes at every step does the same arithmetic whatever the cap
    // (it skips the passes after its own convergence), so only a member that the cap cuts off
    // depends on its batch; such steps are counted (ST_UNCONV), reported per call and per
    // request, and lift the cap to its maximum until the next poll.
    cap = std::min(cap_max, std::max(2, tail ? mx : mx + 1));
    if (short_graph && tail) cap = std::min(cap_max, 1);
    if (!tail && unconv > unconv_seen) cap = cap_max;  // with the tail a cut happens only at max_cycles
    unconv_seen = unconv;
  }
  int start_async(const std::vector<Job*>& J, hipStream_t s) {
    size_t n = 0;
    for (Job* j : J) n += (size_t)j->nmem * STATS_STRIDE;
    if (n > pinned_n) return ENVAR_OK;  // sized by the last synchronous absorb
    if (!ev) HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    size_t o = 0;
    for (Job* j : J) {
      HIP_OK(hipMemcpyAsync(pinned + o, j->w_<double>(j->w.stats), (size_t)j->nmem * STATS_STRIDE * 8,
                            hipMemcpyDeviceToHost, s));
      o += (size_t)j->nmem * STATS_STRIDE;
    }
    HIP_OK(hipEventRecord(ev, s));
    pending = true;
    watched_n = n;
    return ENVAR_OK;
  }
  size_t watched_n = 0;
  void poll() {
    if (pending && hipEventQuery(ev) == hipSuccess) {
      absorb(watched_n);
      pending = false;
    }
  }
  void drain() {
    if (pending) {
      (void)hipEventSynchronize(ev);
      pending = false;
    }
  }

  // Advance every job by one step. `fresh` = some job is at its first step
  // (eager launch followed by an exact cap calibration).
  template <typename TT>
  int step(std::vector<Job*>& J, hipStream_t s, Timer* tm, int steps_left_min, bool use_graphs) {
    bool fresh = false;
    tail = true;
    short_graph = false;
    for (Job* j : J) {
      fresh = fresh || j->step == 0;
      tail = tail && tail_fits(*j) && !(j->P.p.flags & ENVAR_FLAG_NO_TAIL);
      short_graph = short_graph || (j->P.p.flags & ENVAR_FLAG_SHORT_GRAPH);
    }
    const bool sampled = tm && tm->cur >= 0;
    const int par = J[0]->step & 1;
    int rc;
    if (!fresh && !sampled && use_graphs && steps_left_min >= 16) {
      const long key = epoch * 1024 + cap;
      if (G.key[par] != key) {
        G.drop(par);
        if (!G.cs) HIP_OK(hipStreamCreateWithFlags(&G.cs, hipStreamNonBlocking));
        HIP_OK(hipStreamBeginCapture(G.cs, hipStreamCaptureModeThreadLocal));
        rc = batch_step<TT>(J, G.cs, cap, tail, nullptr);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(G.cs, &g);
        if (rc) {
          if (g) (void)hipGraphDestroy(g);
          return rc;
        }
        if (ec != hipSuccess) return fail(ENVAR_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
        G.g[par] = g;
        HIP_OK(hipGraphInstantiate(&G.x[par], g, nullptr, nullptr, 0));
        G.key[par] = key;
      }
      G.ls = s;  // a Driver replays on one stream; retired executables wait on it
      HIP_OK(hipGraphLaunch(G.x[par], s));
    } else {
      // a job's first step runs with the largest cap, whatever the batch needed lately (the step
      // that switches its forcing on can need more passes than any step before it): a request
      // that joins a running batch starts like a forward of its own
      rc = batch_step<TT>(J, s, fresh ? std::max(cap, cap_max) : cap, tail, sampled ? tm : nullptr);
      if (rc) return rc;
    }
    for (Job* j : J) {
      j->last_cur = j->step & 1;
      ++j->step;
    }
    if (fresh) return absorb_now(J, s);
    const int s0 = J[0]->step;
    if (s0 % 16 == 0) {
      poll();
      if (!pending) return start_async(J, s);
    }
    return ENVAR_OK;
  }
};

static int collect_stats(const Plan& P, const WS& w, void* ws, int nmem, hipStream_t s, envar_stats* st,
                         const double* J_dev) {
  std::vector<double> h((size_t)nmem * STATS_STRIDE), dm(nmem), J(nmem);
  HIP_OK(hipMemcpyAsync(h.data(), at<double>(ws, w.stats), h.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(dm.data(), at<double>(ws, w.divmax), dm.size() * 8, hipMemcpyDeviceToHost, s));
  if (J_dev) HIP_OK(hipMemcpyAsync(J.data(), J_dev, J.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  std::memset(st, 0, sizeof *st);
  double cyc = 0.0, steps = 0.0;
  for (int i = 0; i < nmem; ++i) {
    const double* r = &h[(size_t)i * STATS_STRIDE];
    cyc += r[ST_CYCLES];
    steps += r[ST_STEPS];
    st->max_cycles_used = std::max(st->max_cycles_used, (int)r[ST_MAXCYC]);
    st->unconverged += (int)r[ST_UNCONV];
    st->max_resid = std::max(st->max_resid, r[ST_MAXRES]);
    if (!(r[ST_MAXRES] == r[ST_MAXRES])) st->max_resid = NAN;
    st->max_div = std::max(st->max_div, dm[i]);
    if (!(dm[i] == dm[i])) st->max_div = NAN;
    if (J_dev && !std::isfinite(J[i])) st->diverged += 1;
  }
  st->mean_cycles = steps > 0 ? cyc / steps : 0.0;
  st->steps = nmem > 0 ? (int)(steps / nmem) : 0;
  st->cell_steps = (double)P.ncells * steps;
  return ENVAR_OK;
}

}  // namespace envar

using namespace envar;

// ============================================================================ C ABI
extern "C" {

const char* envar_last_error(void) { return g_err.c_str(); }
const char* envar_version(void) { return "envar-mi355x 0.1 (gfx950)"; }

int envar_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream) {
  if (!src_dev || !dst_dev || bytes % 16 != 0) return fail(ENVAR_EINVAL, "16-byte multiple and non-NULL buffers required");
  if (((uintptr_t)src_dev | (uintptr_t)dst_dev) & 15) return fail(ENVAR_EINVAL, "buffers must be 16-byte aligned");
  launch_stream_copy(src_dev, dst_dev, (long)(bytes / 16), (hipStream_t)stream);
  HIP_OK(hipGetLastError());
  return ENVAR_OK;
}

int envar_control_dim(const envar_problem* p, int64_t* m) {
  Plan P;
  int rc = make_plan(p, P);
  if (rc) return rc;
  if (!m) return fail(ENVAR_EINVAL, "m is NULL");
  *m = P.m;
  return ENVAR_OK;
}

int envar_cell_count(const envar_problem* p, int64_t* ncells) {
  Plan P;
  int rc = make_plan(p, P);
  if (rc) return rc;
  if (!ncells) return fail(ENVAR_EINVAL, "ncells is NULL");
  *ncells = P.ncells;
  return ENVAR_OK;
}

size_t envar_state_bytes(const envar_problem* p) {
  Plan P;
  if (make_plan(p, P)) return 0;
  return P.s_total;
}

size_t envar_workspace_bytes(const envar_problem* p, int32_t n_rows) {
  Plan P;
  if (make_plan(p, P) || n_rows < 1) return 0;
  return make_ws(P, n_rows).total;
}

int envar_state_init(const envar_problem* p, const double* u, const double* v, const double* tu_prev,
                     const double* tv_prev, const double* phi, void* state_dev, void* stream) {
  Plan P;
  int rc = make_plan(p, P);
  if (rc) return rc;
  if (!u || !v || !state_dev) return fail(ENVAR_EINVAL, "u, v and state_dev are required");
  if ((tu_prev == nullptr) != (tv_prev == nullptr)) return fail(ENVAR_EINVAL, "tu_prev and tv_prev go together");
  hipStream_t s = (hipStream_t)stream;
  const Geo& g = P.lev[0];
  const long pl = g.plane();
  const int NX = g.nx, NY = g.ny;
  std::vector<double> bu(pl, 0.0), bv(pl, 0.0), btu(pl, 0.0), btv(pl, 0.0), bphi(pl, 0.0);
  const double y0 = p->geometry == ENVAR_CHANNEL ? 0.0 : -1.0;
  const bool uniform = p->geometry == ENVAR_CAVITY_PAPER;  // the paper geometry's uniform inflow
  for (int j = 0; j < NY; ++j)
    for (int i = 0; i <= NX; ++i) {
      const bool w = g.fluid(i - 1, j), e = g.fluid(i, j);
      double val = 0.0;
      if (w && e) val = u[(size_t)j * (NX + 1) + i];
      else if (i == NX && w) val = u[(size_t)j * (NX + 1) + i];
      else if (i == 0 && e) {
        const double y = y0 + (j + 0.5) * g.h;
        val = uniform ? 1.0 : 4.0 * y * (1.0 - y);
      }
      if (!std::isfinite(val)) return fail(ENVAR_EINVAL, "non-finite u at (%d, %d)", i, j);
      bu[g.at(i, j)] = val;
      if (tu_prev && w && e) btu[g.at(i, j)] = tu_prev[(size_t)j * (NX + 1) + i];
    }
  for (int j = 0; j <= NY; ++j)
    for (int i = 0; i < NX; ++i) {
      const bool sfl = g.fluid(i, j - 1), nfl = g.fluid(i, j);
      double val = (sfl && nfl) ? v[(size_t)j * NX + i] : 0.0;
      if (!std::isfinite(val)) return fail(ENVAR_EINVAL, "non-finite v at (%d, %d)", i, j);
      bv[g.at(i, j)] = val;
      if (tv_prev && sfl && nfl) btv[g.at(i, j)] = tv_prev[(size_t)j * NX + i];
    }
  if (phi)
    for (int j = 0; j < NY; ++j)
      for (int i = 0; i < NX; ++i)
        if (g.fluid(i, j)) bphi[g.at(i, j)] = phi[(size_t)j * NX + i];
  std::vector<int> cmap(pl, -1);
  for (size_t k = 0; k < P.ctrl_cells.size(); ++k) {
    const int c = P.ctrl_cells[k];
    cmap[g.at(c % NX, c / NX)] = (int)k;
  }
  Geo gc = P.lev[P.nlev_grid];
  for (int l = 1; l < P.ncoarse; ++l) gc = gc.coarser();
  std::vector<double> ainv;
  std::vector<int> aidx;
  coarse_inverse(gc, ainv, aidx);
  {
    const size_t nc = aidx.size();
    std::vector<double> t(ainv.size());
    for (size_t q = 0; q < nc; ++q)
      for (size_t r = 0; r < nc; ++r) t[r * nc + q] = ainv[q * nc + r];
    ainv.swap(t);  // the coarse kernel reads the transpose
  }
  // Poisson diagonal codes of the tiled levels and the first LDS level
  std::vector<std::vector<unsigned char>> codes(P.nlev_grid + 1);
  for (int l = 0; l <= P.nlev_grid; ++l) {
    const Geo& gl = P.lev[l];
    codes[l].assign(gl.plane(), 0);
    for (int j = 0; j < gl.ny; ++j)
      for (int i = 0; i < gl.nx; ++i)
        if (gl.fluid(i, j)) codes[l][gl.at(i, j)] = (unsigned char)gl.diag_count(i, j);
  }
  int meta[64] = {0};
  meta[0] = tu_prev ? 0 : 1;  // cold start flag
  char* S = (char*)state_dev;
  HIP_OK(hipMemsetAsync(S, 0, P.s_total, s));
  HIP_OK(hipMemcpyAsync(S + P.s_meta, meta, sizeof meta, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(S + P.s_u, bu.data(), pl * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(S + P.s_v, bv.data(), pl * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(S + P.s_tu, btu.data(), pl * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(S + P.s_tv, btv.data(), pl * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(S + P.s_phi, bphi.data(), pl * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(S + P.s_cmap, cmap.data(), pl * 4, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(S + P.s_ainv, ainv.data(), ainv.size() * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(S + P.s_aidx, aidx.data(), aidx.size() * 4, hipMemcpyHostToDevice, s));
  for (int l = 0; l <= P.nlev_grid; ++l)
    HIP_OK(hipMemcpyAsync(S + P.s_code[l], codes[l].data(), codes[l].size(), hipMemcpyHostToDevice, s));
  launch_shift(g, at<double>(state_dev, P.s_u), at<double>(state_dev, P.s_v), at<double>(state_dev, P.s_shu),
               at<double>(state_dev, P.s_shv), s);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(s));
  return ENVAR_OK;
}

int envar_state_read(const envar_problem* p, const void* state_dev, double* u, double* v, double* tu_prev,
                     double* tv_prev, double* phi) {
  Plan P;
  int rc = make_plan(p, P);
  if (rc) return rc;
  if (!state_dev) return fail(ENVAR_EINVAL, "state_dev is NULL");
  const Geo& g = P.lev[0];
  const size_t pb = (size_t)g.pitch * 8;
  const char* S = (const char*)state_dev;
  if (u) HIP_OK(hipMemcpy2D(u, (g.nx + 1) * 8, S + P.s_u, pb, (g.nx + 1) * 8, g.ny, hipMemcpyDeviceToHost));
  if (v) HIP_OK(hipMemcpy2D(v, g.nx * 8, S + P.s_v, pb, g.nx * 8, g.ny + 1, hipMemcpyDeviceToHost));
  if (tu_prev)
    HIP_OK(hipMemcpy2D(tu_prev, (g.nx + 1) * 8, S + P.s_tu, pb, (g.nx + 1) * 8, g.ny, hipMemcpyDeviceToHost));
  if (tv_prev) HIP_OK(hipMemcpy2D(tv_prev, g.nx * 8, S + P.s_tv, pb, g.nx * 8, g.ny + 1, hipMemcpyDeviceToHost));
  if (phi) HIP_OK(hipMemcpy2D(phi, g.nx * 8, S + P.s_phi, pb, g.nx * 8, g.ny, hipMemcpyDeviceToHost));
  return ENVAR_OK;
}

}  // extern "C"

namespace envar {

struct JobOut {
  double* J = nullptr;
  double* fields = nullptr;
  bool spinup_store = false;
};

// ---------------------------------------------------------------------------- tile tuner
// Chooses the tile height (8 or 16 rows) of the predictor, the projection and
// each tiled multigrid level by timing both candidates with HIP events on the
// job's own workspace, before its members are initialised (the trial launches
// only write workspace buffers that the initialisation or the first step
// rewrites). No launch in the trial depends on the convergence slots: the
// multigrid trials run as the first pass of a cycle. Every candidate gives
// bitwise the same results, so the choice only affects speed. Choices are kept
// per (grid, geometry, precision, member count rounded up to a power of two).
struct TileChoice {
  int pred = 8, proj = 8;
  int mg[MAX_LEVELS] = {16, 16, 16, 16, 16, 16, 16, 16, 16, 16, 16, 16};
};
static std::mutex g_tune_mu;
static std::map<std::array<int, 4>, TileChoice> g_tune;

static void apply_choice(Job& j, const TileChoice& c) {
  j.rows_pred = c.pred;
  j.rows_proj = c.proj;
  for (int l = 0; l < MAX_LEVELS; ++l) j.rows_mg[l] = c.mg[l];
}

template <typename TT>
static int tune_job(Job& j, hipStream_t s) {
  typedef TT T;
  const Plan& P = j.P;
  const int fl = P.p.flags;
  TileChoice c;
  if (fl & (ENVAR_FLAG_TILES_8 | ENVAR_FLAG_TILES_16 | ENVAR_FLAG_TILES_32)) {
    const int r = (fl & ENVAR_FLAG_TILES_32) ? 32 : (fl & ENVAR_FLAG_TILES_16) ? 16 : 8;
    c.pred = c.proj = (r >= 16 && P.rows16) ? 16 : 8;
    for (int l = 0; l < MAX_LEVELS; ++l) c.mg[l] = (r == 32 && l < P.nlev_grid && P.lev[l].jc % 32) ? 16 : r;
    apply_choice(j, c);
    return ENVAR_OK;
  }
  if (fl & ENVAR_FLAG_NO_TUNE) {
    apply_choice(j, c);
    return ENVAR_OK;
  }
  int bucket = 1;
  while (bucket < j.nmem) bucket *= 2;
  const std::array<int, 4> key = {P.n, P.p.geometry, P.mixed, bucket};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      apply_choice(j, it->second);
      return ENVAR_OK;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_OK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ENVAR_EDEVICE, "hipEventCreate failed");
  }
  constexpr int REPS = 10;
  int rc = ENVAR_OK;
  // mean device time of one call of `launch` (after one untimed call)
  auto timed = [&](auto launch) -> float {
    launch();
    float ms = 0.f;
    if (hipEventRecord(e0, s) != hipSuccess) rc = ENVAR_EDEVICE;
    for (int r = 0; r < REPS; ++r) launch();
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      rc = ENVAR_EDEVICE;
    return ms / REPS;
  };
  auto one = [](auto a) {
    auto m = seg_begin<decltype(a)>();
    seg_add(m, a, a.ntiles * a.nmem);
    return m;
  };
  if (P.rows16) {
    // the steady-state kernel: predictor fused with the previous projection
    float t[2];
    for (int v = 0; v < 2; ++v)
      t[v] = timed([&] { launch_predictor<double>(one(pred_args(j, v ? 16 : 8, true)), s); });
    c.pred = c.proj = t[1] < t[0] ? 16 : 8;
  }
  for (int l = 0; l < P.nlev_grid; ++l) {
    const int k = (P.mixed && l == 0) ? 1 : 0;  // a first pass: no launch reads a convergence slot
    // 32-row tiles only where the cavity rows take whole tiles
    const int nv = P.lev[l].jc % 32 == 0 ? 3 : 2;
    float t[3];
    int best = 0;
    for (int v = 0; v < nv; ++v) {
      const int rows = 8 << v;
      t[v] = timed([&] {
        launch_mg_pre<T>(one(pre_args<T>(j, l, k, rows)), s);
        launch_mg_post<T>(one(post_args<T>(j, l, 0, rows)), l > 0 ? POST_PLAIN : P.mixed ? POST_REFINE : POST_NORM, s);
      });
      if (t[v] < 0.97f * t[best]) best = v;  // a taller tile has to win by 3% (timing noise of short launches)
    }
    c.mg[l] = 8 << best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != ENVAR_OK) return fail(rc, "tile tuner: event timing failed");
  HIP_OK(hipGetLastError());
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = c;
  }
  apply_choice(j, c);
  return ENVAR_OK;
}

static void put_rows(const Job& j, envar_stats* st) {
  if (!st) return;
  st->rows_pred = j.rows_pred;
  st->rows_proj = j.rows_proj;
  for (int l = 0; l < 4; ++l) st->rows_mg[l] = l < j.P.nlev_grid ? j.rows_mg[l] : 0;
}

// ---------------------------------------------------------------------------- lanes
// The members of a batch advance in lanes: member groups on separate streams, each with its own
// step graphs and cycle cap. Members are independent over the horizon, so one lane's
// latency-bound phases (the coarse multigrid levels, launches of passes its members skip, the
// gaps between graph nodes) overlap with another lane's bandwidth-bound kernels. A lane runs
// member slices of the batch's jobs: jobs are split into contiguous member ranges of about equal
// work and the slices dealt to the least loaded lane, largest first. Results do not depend on the
// split (per-member convergence; every kernel is per member).
constexpr int LANES_DEFAULT = 2;

struct Unit {
  int job, a, b;  // members [a, b) of jobs[job]
  double work;    // fluid cells x members x steps
};

static std::vector<std::vector<Unit>> make_lanes(const std::vector<Job>& jobs, int nlanes) {
  double W = 0.0;
  std::vector<Unit> units;
  for (const Job& j : jobs) W += (double)j.P.ncells * j.nmem * j.horizon;
  const double target = W / std::max(1, nlanes);
  for (size_t k = 0; k < jobs.size(); ++k) {
    const Job& j = jobs[k];
    const double wj = (double)j.P.ncells * j.nmem * j.horizon;
    int parts = (int)std::lround(wj / std::max(target, 1.0));
    parts = std::max(1, std::min(parts, std::min(j.nmem, nlanes)));
    for (int q = 0; q < parts; ++q) {
      const int a = (int)((long)j.nmem * q / parts), b = (int)((long)j.nmem * (q + 1) / parts);
      units.push_back({(int)k, a, b, (double)j.P.ncells * (b - a) * j.horizon});
    }
  }
  std::stable_sort(units.begin(), units.end(), [](const Unit& x, const Unit& y) { return x.work > y.work; });
  const int L = std::max(1, std::min(nlanes, (int)units.size()));
  std::vector<std::vector<Unit>> lanes(L);
  std::vector<double> load(L, 0.0);
  for (const Unit& u : units) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lanes[l].push_back(u);
    load[l] += u.work;
  }
  return lanes;
}

// members [a, b) of job j (their control rows, sensor series and workspace slices)
static Job slice_job(const Job& j, const WS& stride, int a, int b) {
  Job s = j;
  s.w = slice_ws(j.w, stride, a);
  s.nmem = b - a;
  if (j.ctrl) s.ctrl = j.ctrl + (size_t)a * j.P.m;
  if (j.obs) s.obs = j.obs + (size_t)a * OBS_CHANNELS * j.obs_K;
  return s;
}

// Streams and events of the lanes beyond the first (which runs on the call's stream): created
// once per host thread at default priority and kept for the process.
struct LaneRes {
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  int ensure(int nstreams, int nevents) {
    while ((int)streams.size() < nstreams) {
      hipStream_t q = nullptr;
      HIP_OK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
      streams.push_back(q);
    }
    while ((int)events.size() < nevents) {
      hipEvent_t e = nullptr;
      HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      events.push_back(e);
    }
    return ENVAR_OK;
  }
};
static thread_local LaneRes t_lanes;

// `dst` waits for everything queued so far on `src`
static int stream_after(hipStream_t dst, hipStream_t src, hipEvent_t e) {
  HIP_OK(hipEventRecord(e, src));
  HIP_OK(hipStreamWaitEvent(dst, e, 0));
  return ENVAR_OK;
}

// Integrate every job to its own horizon; jobs leave their lane as they finish. Kernel timing
// (tm) samples the first lane; a sampled step runs with the other lanes held, so that its
// kernels are timed alone.
template <typename TT>
static int run_batch(std::vector<Job>& jobs, const std::vector<JobOut>& outs, hipStream_t s, Timer* tm, bool graphs,
                     int nlanes = 1) {
  const auto plan = make_lanes(jobs, nlanes);
  const int L = (int)plan.size();
  std::vector<std::vector<Job>> lj(L);
  std::vector<std::vector<JobOut>> lo(L);
  int cap_max = 0;
  for (int l = 0; l < L; ++l)
    for (const Unit& u : plan[l]) {
      const Job& j = jobs[u.job];
      JobOut o = outs[u.job];
      if (u.a == 0 && u.b == j.nmem) {
        lj[l].push_back(j);
      } else {
        WS stride;
        (void)make_ws(j.P, j.nmem, &stride);
        lj[l].push_back(slice_job(j, stride, u.a, u.b));
        const Geo& g = j.P.lev[0];
        if (o.J) o.J += u.a;
        if (o.fields) o.fields += (size_t)u.a * ((size_t)g.ny * (g.nx + 1) + (size_t)(g.ny + 1) * g.nx);
        o.spinup_store = false;  // a spin-up has one member and is never split
      }
      lo[l].push_back(o);
      cap_max = std::max(cap_max, j.P.cap_max);
    }
  for (int l = 0; l < L; ++l)
    for (size_t k = 0; k < lj[l].size(); ++k) {
      Job& j = lj[l][k];
      const int rc = tune_job<TT>(j, s);
      if (rc) return rc;
      init_members<TT>(j, s);
      const Unit& u = plan[l][k];
      if (u.a == 0) {  // the job reports the tile heights of the slice that holds its first member
        Job& whole = jobs[u.job];
        whole.rows_pred = j.rows_pred;
        whole.rows_proj = j.rows_proj;
        std::copy(j.rows_mg, j.rows_mg + MAX_LEVELS, whole.rows_mg);
      }
    }
  if (tm) {
    tm->members = 0;
    for (const Job& j : lj[0]) tm->members += j.nmem;
  }
  std::vector<hipStream_t> st(L, s);
  if (L > 1) {
    int rc = t_lanes.ensure(L - 1, 2 * L + 2);
    if (rc) return rc;
    for (int l = 1; l < L; ++l) {
      st[l] = t_lanes.streams[l - 1];
      rc = stream_after(st[l], s, t_lanes.events[l]);  // fork: the lanes start after the set-up
      if (rc) return rc;
    }
  }
  std::vector<std::unique_ptr<Driver>> D(L);
  std::vector<std::vector<Job*>> active(L);
  std::vector<std::vector<int>> which(L);
  for (int l = 0; l < L; ++l) {
    D[l].reset(new Driver);
    D[l]->cap = D[l]->cap_max = cap_max;
    for (size_t k = 0; k < lj[l].size(); ++k) {
      active[l].push_back(&lj[l][k]);
      which[l].push_back((int)k);
    }
  }
  int rc = ENVAR_OK;
  for (bool any = true; any;) {
    any = false;
    for (int l = 0; l < L; ++l) {
      std::vector<Job*>& A = active[l];
      if (A.empty()) continue;
      any = true;
      int left = 1 << 30, longest = 0;
      for (Job* j : A) {
        left = std::min(left, j->horizon - j->step);
        longest = std::max(longest, j->horizon);
      }
      Timer* lt = l == 0 ? tm : nullptr;
      if (lt && lt->begin_step(A[0]->step, longest)) return fail(ENVAR_EDEVICE, "hipEventCreate failed");
      const bool alone = lt && lt->cur >= 0 && L > 1;
      if (alone)  // the sampled step starts after every other lane's queued work ...
        for (int q = 1; q < L && !rc; ++q) rc = stream_after(st[0], st[q], t_lanes.events[L + q]);
      if (!rc) rc = D[l]->step<TT>(A, st[l], lt, left, graphs);
      if (alone)  // ... and the other lanes continue after it
        for (int q = 1; q < L && !rc; ++q) rc = stream_after(st[q], st[0], t_lanes.events[0]);
      if (rc) return rc;
      bool changed = false;
      for (size_t k = 0; k < A.size();) {
        if (A[k]->step >= A[k]->horizon) {
          const JobOut& o = lo[l][which[l][k]];
          finish_job(*A[k], o.J, o.fields, o.spinup_store, st[l]);
          A.erase(A.begin() + k);
          which[l].erase(which[l].begin() + k);
          changed = true;
        } else {
          ++k;
        }
      }
      if (changed) ++D[l]->epoch;
    }
  }
  for (int l = 1; l < L && !rc; ++l) rc = stream_after(s, st[l], t_lanes.events[L + l]);  // join
  for (auto& d : D) d->drain();
  if (rc) return rc;
  HIP_OK(hipGetLastError());
  return ENVAR_OK;
}

static void fill_timer_stats(Timer& timer, envar_stats* stats, int n_rows) {
  if (!timer.on || timer.samples == 0) return;
  double* outs[TM_N] = {&stats->predictor_us, &stats->pre_us, &stats->post_us,
                        &stats->resid_us, &stats->project_us, &stats->vcycle_us};
  for (int t = 0; t < TM_N; ++t) {
    double sum = 0.0;
    int cnt = 0;
    for (int q = 0; q < timer.samples; ++q) {
      if (!timer.recorded(q, t)) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, timer.ev[((size_t)q * TM_N + t) * 2], timer.ev[((size_t)q * TM_N + t) * 2 + 1]) ==
          hipSuccess) {
        sum += ms;
        ++cnt;
      }
    }
    *outs[t] = cnt ? 1e3 * sum / cnt : 0.0;
  }
  stats->timed_steps = timer.samples;
  stats->timed_members = timer.members > 0 ? timer.members : n_rows;
  (void)hipGetLastError();  // the event queries leave no sticky error behind
}

static int make_job(const Plan& P, const void* state_dev, const double* controls_dev, int n_rows, int horizon,
                    void* ws_dev, size_t ws_bytes, Job& j) {
  j.P = P;
  j.w = make_ws(P, n_rows);
  if (ws_bytes < j.w.total) return fail(ENVAR_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, j.w.total);
  j.ws = ws_dev;
  j.state = state_dev;
  j.ctrl = controls_dev;
  j.nmem = n_rows;
  j.horizon = horizon;
  j.step = 0;
  return ENVAR_OK;
}

static int forward_impl(const Plan& P, const void* state_dev, const double* controls_dev, int n_rows, int horizon,
                        void* ws_dev, size_t ws_bytes, double* J_dev, double* fields_dev, envar_stats* stats,
                        hipStream_t s, bool spinup_store, double* obs_dev = nullptr, int obs_every = 1) {
  std::vector<Job> jobs(1);
  int rc = make_job(P, state_dev, controls_dev, n_rows, horizon, ws_dev, ws_bytes, jobs[0]);
  if (rc) return rc;
  if (obs_dev) {
    jobs[0].obs = obs_dev;
    jobs[0].obs_every = obs_every;
    jobs[0].obs_K = horizon / obs_every;
  }
  std::vector<JobOut> outs(1);
  outs[0].J = J_dev;
  outs[0].fields = fields_dev;
  outs[0].spinup_store = spinup_store;
  Timer timer;
  timer.on = stats != nullptr && (P.p.flags & ENVAR_FLAG_TIME_KERNELS);
  timer.every = std::max(1, (horizon - 1 + timer.max_samples - 1) / timer.max_samples);
  const bool graphs = !(P.p.flags & ENVAR_FLAG_NO_GRAPHS);
  const int nl = (P.p.flags & ENVAR_FLAG_ONE_LANE) ? 1 : LANES_DEFAULT;
  rc = P.mixed ? run_batch<float>(jobs, outs, s, timer.on ? &timer : nullptr, graphs, nl)
               : run_batch<double>(jobs, outs, s, timer.on ? &timer : nullptr, graphs, nl);
  if (rc) return rc;
  if (stats) {
    rc = collect_stats(P, jobs[0].w, ws_dev, n_rows, s, stats, J_dev);
    put_rows(jobs[0], stats);
    if (rc) return rc;
    fill_timer_stats(timer, stats, n_rows);
    if (stats->diverged > 0) return fail(ENVAR_EDIVERGED, "%d member(s) produced a non-finite cost", stats->diverged);
  }
  return ENVAR_OK;
}

}  // namespace envar

extern "C" {

int envar_forward_batch(envar_job* jobs_in, int32_t njobs, void* stream) {
  if (!jobs_in || njobs < 1 || njobs > MAX_SEG) return fail(ENVAR_EINVAL, "njobs must be in [1, %d]", MAX_SEG);
  hipStream_t s = (hipStream_t)stream;
  std::vector<Job> jobs(njobs);
  std::vector<JobOut> outs(njobs);
  int prec = -1;
  bool graphs = true, one_lane = false;
  for (int k = 0; k < njobs; ++k) {
    envar_job& q = jobs_in[k];
    Plan P;
    int rc = make_plan(&q.problem, P);
    if (rc) return rc;
    if (prec < 0) prec = P.mixed;
    if (P.mixed != prec) return fail(ENVAR_EINVAL, "all jobs of a batch must share one precision");
    if (!q.state_dev || !q.ws_dev || !q.J_dev || !q.controls_dev) return fail(ENVAR_EINVAL, "job %d: NULL pointer", k);
    if (q.n_rows < 1 || q.horizon < 1) return fail(ENVAR_EINVAL, "job %d: n_rows and horizon must be >= 1", k);
    if (q.m != P.m) return fail(ENVAR_EINVAL, "job %d: m = %lld but the control region has m = %ld", k,
                                (long long)q.m, P.m);
    rc = make_job(P, q.state_dev, q.controls_dev, q.n_rows, q.horizon, q.ws_dev, q.ws_bytes, jobs[k]);
    if (rc) return rc;
    outs[k].J = q.J_dev;
    outs[k].fields = q.fields_dev;
    graphs = graphs && !(P.p.flags & ENVAR_FLAG_NO_GRAPHS);
    one_lane = one_lane || (P.p.flags & ENVAR_FLAG_ONE_LANE);
  }
  const int nl = one_lane ? 1 : LANES_DEFAULT;
  int rc = prec ? run_batch<float>(jobs, outs, s, nullptr, graphs, nl)
                : run_batch<double>(jobs, outs, s, nullptr, graphs, nl);
  if (rc) return rc;
  int diverged = 0;
  for (int k = 0; k < njobs; ++k)
    if (jobs_in[k].stats) {
      rc = collect_stats(jobs[k].P, jobs[k].w, jobs[k].ws, jobs[k].nmem, s, jobs_in[k].stats, jobs_in[k].J_dev);
      put_rows(jobs[k], jobs_in[k].stats);
      if (rc) return rc;
      diverged += jobs_in[k].stats->diverged;
    }
  if (diverged > 0) return fail(ENVAR_EDIVERGED, "%d member(s) produced a non-finite cost", diverged);
  return ENVAR_OK;
}

int envar_spinup(const envar_problem* p, void* state_dev, int32_t steps, void* ws_dev, size_t ws_bytes,
                 envar_stats* stats, void* stream) {
  Plan P;
  int rc = make_plan(p, P);
  if (rc) return rc;
  if (!state_dev || !ws_dev) return fail(ENVAR_EINVAL, "state_dev and ws_dev are required");
  if (steps < 1) return fail(ENVAR_EINVAL, "steps must be >= 1");
  return forward_impl(P, state_dev, nullptr, 1, steps, ws_dev, ws_bytes, nullptr, nullptr, stats,
                      (hipStream_t)stream, true);
}

int envar_forward(const envar_problem* p, const void* state_dev, const double* controls_dev, int32_t n_rows,
                  int64_t m, int32_t horizon, void* ws_dev, size_t ws_bytes, double* J_dev, double* fields_dev,
                  envar_stats* stats, void* stream) {
  Plan P;
  int rc = make_plan(p, P);
  if (rc) return rc;
  if (!state_dev || !ws_dev || !J_dev || !controls_dev) return fail(ENVAR_EINVAL, "NULL device pointer");
  if (n_rows < 1) return fail(ENVAR_EINVAL, "n_rows must be >= 1");
  if (m != P.m) return fail(ENVAR_EINVAL, "m = %lld but the control region has m = %ld", (long long)m, P.m);
  if (horizon < 1) return fail(ENVAR_EINVAL, "horizon must be >= 1");
  return forward_impl(P, state_dev, controls_dev, n_rows, horizon, ws_dev, ws_bytes, J_dev, fields_dev, stats,
                      (hipStream_t)stream, false);
}

int envar_forward_obs(const envar_problem* p, const void* state_dev, const double* controls_dev, int32_t n_rows,
                      int64_t m, int32_t horizon, int32_t every, void* ws_dev, size_t ws_bytes, double* J_dev,
                      double* obs_dev, envar_stats* stats, void* stream) {
  Plan P;
  int rc = make_plan(p, P);
  if (rc) return rc;
  if (!state_dev || !ws_dev || !J_dev || !controls_dev || !obs_dev) return fail(ENVAR_EINVAL, "NULL device pointer");
  if (n_rows < 1) return fail(ENVAR_EINVAL, "n_rows must be >= 1");
  if (m != P.m) return fail(ENVAR_EINVAL, "m = %lld but the control region has m = %ld", (long long)m, P.m);
  if (horizon < 1) return fail(ENVAR_EINVAL, "horizon must be >= 1");
  if (every < 1 || horizon / every < 1) return fail(ENVAR_EINVAL, "every must be in [1, horizon]");
  if (!P.obs_ok) return fail(ENVAR_EINVAL, "the lid sensors need the cavity geometry");
  return forward_impl(P, state_dev, controls_dev, n_rows, horizon, ws_dev, ws_bytes, J_dev, nullptr, stats,
                      (hipStream_t)stream, false, obs_dev, every);
}

}  // extern "C"

// ---------------------------------------------------------------------------- gradient
namespace envar {
struct GradLayout {
  size_t X, Xt, dJ, rhs, partial, tmp, G, c, info, W, Wt, ev, jscr, total;
  int nsplit, dim;
  long kchunk;
  // the split of an FP64 Gram (the FP64 path's own, which the mixed path's FP64 re-solve takes so
  // that it forms bitwise the FP64 path's Gram)
  int nsplit64;
  long kchunk64;
};
constexpr int GRAD_PINV_MAX = 512;  // largest system the pseudo-inverse (one-workgroup Jacobi) takes
constexpr double GRAD_PINV_RCOND = 1e-12;

static GradLayout grad_layout(int n, long m, int precision) {
  GradLayout L{};
  const size_t xs = precision == ENVAR_MIXED ? 4 : 8;
  const bool tall = n <= m;
  L.dim = tall ? n : (int)m;
  const long klen = tall ? m : n;  // contraction length
  gram_split(L.dim, klen, (int)xs, L.nsplit, L.kchunk);
  gram_split(L.dim, klen, 8, L.nsplit64, L.kchunk64);
  const size_t nsp = (size_t)std::max(L.nsplit, L.nsplit64);
  const size_t ngr = (size_t)std::max(gram_reduce_groups(L.nsplit), gram_reduce_groups(L.nsplit64));
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t a = o;
    o = align256(o + b);
    return a;
  };
  // FP64 with n <= m stores no anomalies: the Gram and the final product form them from the
  // control rows (L.X is then not used)
  L.X = precision == ENVAR_FP64 && tall ? 0 : take((size_t)n * m * xs);
  L.Xt = tall ? 0 : take((size_t)n * m * xs);
  L.dJ = take((size_t)n * 8);
  L.rhs = take((size_t)L.dim * 8);
  L.partial = take(nsp * L.dim * L.dim * 8);
  L.tmp = take(ngr * L.dim * L.dim * 8);
  L.G = take((size_t)L.dim * L.dim * 8);
  L.c = take((size_t)L.dim * 8);
  L.info = take(256);
  if (L.dim <= GRAD_PINV_MAX) {  // the pseudo-inverse: eigenvectors, eigenvalues, Jacobi's matrices
    const size_t d = (size_t)L.dim, ne = d + (d & 1);
    L.W = take(d * d * 8);
    L.Wt = take(d * d * 8);
    L.ev = take(d * 8);
    L.jscr = take(2 * ne * (ne + 1) * 8);
  }
  L.total = o;
  return L;
}

}  // namespace envar

extern "C" size_t envar_gradient_bytes(int32_t n, int64_t m, int32_t precision) {
  if (n < 1 || m < 1) return 0;
  return grad_layout(n, m, precision & ~ENVAR_GRADIENT_PINV).total;
}

namespace envar {
// pinned_flag: read the solve's status word through a pinned word of this host thread (allocated
// on the thread's first call and kept); otherwise through pageable memory (no allocation)
template <typename TX>
static int gradient_impl(const double* ctrl, const double* J, int n, long m, int precision, void* ws, double* g,
                         hipStream_t s, bool pinned_flag = true) {
  const bool pinv = (precision & ENVAR_GRADIENT_PINV) != 0;
  precision &= ~ENVAR_GRADIENT_PINV;
  const GradLayout L = grad_layout(n, m, precision);
  const bool tall = n <= m;
  // FP64 rows over at least as many controls as members: the Gram and the final product form the
  // anomalies from the control rows where they read them (the values k_anomaly would store, so the
  // result is the same bit for bit), which saves writing X, reading it back and its workspace.
  // Control rows that are not 16-byte aligned are read element by element.
  const bool fp32 = sizeof(TX) == sizeof(float);
  const bool onfly = !fp32 && tall;
  TX* X = onfly ? nullptr : at<TX>(ws, L.X);  // the workspace holds no X then
  double* dJ = at<double>(ws, L.dJ);
  double* G = at<double>(ws, L.G);
  double* partial = at<double>(ws, L.partial);
  double* rhs = at<double>(ws, L.rhs);
  double* c = at<double>(ws, L.c);
  int* info_dev = at<int>(ws, L.info);
  // the solve's status word, read through a pinned word of this host thread (allocated once, kept
  // for the process) or, for callers that cannot allocate, through pageable memory
  auto read_info = [&](int& info) -> int {
    if (pinned_flag) {
      static thread_local int* flag = nullptr;
      if (!flag) HIP_OK(hipHostMalloc((void**)&flag, sizeof(int), hipHostMallocDefault));
      HIP_OK(hipMemcpyAsync(flag, info_dev, sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      info = *flag;
    } else {
      HIP_OK(hipMemcpyAsync(&info, info_dev, sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
    }
    return ENVAR_OK;
  };
  if (onfly)
    launch_cost_anomaly(J, n, dJ, s);
  else
    launch_anomaly<TX>(ctrl, J, n, m, X, dJ, s);
  if (tall) {
    if (onfly)
      launch_gram_anom(ctrl, n, m, partial, L.nsplit, L.kchunk, s);
    else
      launch_gram<TX>(X, n, m, m, partial, L.nsplit, L.kchunk, s);
    launch_gram_reduce(partial, n, L.nsplit, at<double>(ws, L.tmp), G, s);
    if (!pinv) {
      if (launch_chol_solve(G, dJ, n, c, (double*)info_dev, s)) return fail(ENVAR_EDEVICE, "Cholesky launch failed (n = %d)", n);
      if (onfly)
        launch_gemv_anom(ctrl, n, m, c, g, s);
      else
        launch_gemv_t<TX>(X, n, m, m, c, g, s);
    }
  } else {
    TX* Xt = at<TX>(ws, L.Xt);
    launch_transpose<TX>(X, n, m, Xt, s);
    launch_gram<TX>(Xt, (int)m, n, n, partial, L.nsplit, L.kchunk, s);
    launch_gram_reduce(partial, (int)m, L.nsplit, at<double>(ws, L.tmp), G, s);
    launch_gemv_t<TX>(X, n, m, m, dJ, rhs, s);
    if (!pinv && launch_chol_solve(G, rhs, (int)m, g, (double*)info_dev, s))
      return fail(ENVAR_EDEVICE, "Cholesky launch failed (m = %ld)", m);
  }
  HIP_OK(hipGetLastError());
  int info = 0;
  if (!pinv) {
    // a pivot that is not positive after the ridge or a non-finite solution (a non-finite cost)
    // is not returned as a gradient: the solve leaves both in one word
    const int rc = read_info(info);
    if (rc) return rc;
    if (info < 0) return fail(ENVAR_EDIVERGED, "non-finite least-squares solution (a cost is not finite?)");
    if (info == 0) return ENVAR_OK;
  }
  // A failed factor (or a requested pseudo-inverse). With FP32 anomalies, the Gram's rounding
  // (about 1e-7 of its largest entries) can make the Gram of a nearly dependent ensemble
  // indefinite; the system is then formed again in FP64 from the control rows, the anomalies
  // taken on the fly, which is the FP64 gradient's own arithmetic. A factor that fails in FP64
  // (or the pseudo-inverse asked for) goes to the eigen-pseudo-inverse of the Gram: its
  // eigenvalues at or below 1e-12 of the largest dropped, the minimum-norm solution.
  if (fp32) {
    if (!tall)
      return fail(ENVAR_EDIVERGED, "the FP32 Gram of %d members over %ld controls is not positive definite (pivot %d); "
                  "use ENVAR_FP64", n, m, info);
    launch_gram_anom(ctrl, n, m, partial, L.nsplit64, L.kchunk64, s);
    launch_gram_reduce(partial, n, L.nsplit64, at<double>(ws, L.tmp), G, s);
    if (!pinv) {
      if (launch_chol_solve(G, dJ, n, c, (double*)info_dev, s)) return fail(ENVAR_EDEVICE, "Cholesky launch failed (n = %d)", n);
      HIP_OK(hipGetLastError());
      const int rc = read_info(info);
      if (rc) return rc;
      if (info < 0) return fail(ENVAR_EDIVERGED, "non-finite least-squares solution (a cost is not finite?)");
      if (info == 0) {
        launch_gemv_anom(ctrl, n, m, c, g, s);
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(s));
        return ENVAR_OK;
      }
    }
  }
  if (L.dim > GRAD_PINV_MAX)
    return fail(ENVAR_EDIVERGED, "the ensemble Gram is not positive definite (pivot %d); the pseudo-inverse takes "
                "systems up to %d", info, GRAD_PINV_MAX);
  if (!pinv)  // the failed factor overwrote the Gram: reduce the partials (of an FP64 Gram) again
    launch_gram_reduce(partial, L.dim, L.nsplit64, at<double>(ws, L.tmp), G, s);
  double* W = at<double>(ws, L.W);
  double* ev = at<double>(ws, L.ev);
  if (launch_jacobi(G, L.dim, L.dim, ev, W, at<double>(ws, L.Wt), at<double>(ws, L.jscr), s))
    return fail(ENVAR_EDEVICE, "Jacobi launch failed (n = %d)", L.dim);
  if (launch_pinv_apply(W, ev, L.dim, tall ? dJ : rhs, tall ? c : g, GRAD_PINV_RCOND, info_dev, s))
    return fail(ENVAR_EDEVICE, "pseudo-inverse launch failed (n = %d)", L.dim);
  if (tall) {
    if (fp32 || onfly)
      launch_gemv_anom(ctrl, n, m, c, g, s);
    else
      launch_gemv_t<TX>(X, n, m, m, c, g, s);
  }
  HIP_OK(hipGetLastError());
  const int rc = read_info(info);
  if (rc) return rc;
  if (info != 0) return fail(ENVAR_EDIVERGED, "non-finite pseudo-inverse solution (a cost is not finite?)");
  return ENVAR_OK;
}

}  // namespace envar

extern "C" int envar_gradient(const double* controls_dev, const double* J_dev, int32_t n, int64_t m, int32_t precision,
                   void* ws_dev, size_t ws_bytes, double* g_dev, void* stream) {
  if (n < 1 || m < 1) return fail(ENVAR_EINVAL, "n and m must be >= 1");
  if (!controls_dev || !J_dev || !ws_dev || !g_dev) return fail(ENVAR_EINVAL, "NULL device pointer");
  const int base = precision & ~ENVAR_GRADIENT_PINV;
  if (base != ENVAR_FP64 && base != ENVAR_MIXED) return fail(ENVAR_EINVAL, "unknown precision");
  if (std::min<long>(n, m) > 1024) return fail(ENVAR_EINVAL, "min(n, m) = %ld exceeds 1024", std::min<long>(n, m));
  const GradLayout L = grad_layout(n, m, base);
  if (ws_bytes < L.total) return fail(ENVAR_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
  if (base == ENVAR_MIXED)
    return gradient_impl<float>(controls_dev, J_dev, n, m, precision, ws_dev, g_dev, (hipStream_t)stream);
  return gradient_impl<double>(controls_dev, J_dev, n, m, precision, ws_dev, g_dev, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------- gradient without allocation
// envar_gradient for callers that cannot allocate (code under HIP graph capture, serving loops,
// harnesses that forbid allocation): the workspace is this file-scope device array, one copy per
// GPU, held until the process ends. Host code never passes the array's name to a kernel or a
// copy (on the host it is a stand-in, not a device address): each device's address comes from
// hipGetSymbolAddress, taken once per device with that device current.
namespace envar {
static __device__ __align__(256) unsigned char scratch[ENVAR_GRADIENT_STATIC_MAX_BYTES];
constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[SCRATCH_MAX_DEVICES];

static int scratch_address(void** out) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(ENVAR_EDEVICE, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ENVAR_EDEVICE, "hipGetSymbolAddress returned NULL for the gradient scratch");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return ENVAR_OK;
}
}  // namespace envar

extern "C" int envar_gradient_static(const double* controls_dev, const double* J_dev, int32_t n, int64_t m,
                                     int32_t precision, double* g_dev, void* stream) {
  if (n < 1 || m < 1) return fail(ENVAR_EINVAL, "n and m must be >= 1");
  if (!controls_dev || !J_dev || !g_dev) return fail(ENVAR_EINVAL, "NULL device pointer");
  const int base = precision & ~ENVAR_GRADIENT_PINV;
  if (base != ENVAR_FP64 && base != ENVAR_MIXED) return fail(ENVAR_EINVAL, "unknown precision");
  if (std::min<long>(n, m) > 1024) return fail(ENVAR_EINVAL, "min(n, m) = %ld exceeds 1024", std::min<long>(n, m));
  const GradLayout L = grad_layout(n, m, base);
  if (L.total > ENVAR_GRADIENT_STATIC_MAX_BYTES)
    return fail(ENVAR_ENOMEM, "n = %d, m = %lld needs %zu bytes of scratch; the static array holds %zu", n,
                (long long)m, L.total, (size_t)ENVAR_GRADIENT_STATIC_MAX_BYTES);
  void* ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc) return rc;
  if (base == ENVAR_MIXED)
    return gradient_impl<float>(controls_dev, J_dev, n, m, precision, ws, g_dev, (hipStream_t)stream, false);
  return gradient_impl<double>(controls_dev, J_dev, n, m, precision, ws, g_dev, (hipStream_t)stream, false);
}

// ---------------------------------------------------------------------------- vector-observation EnVar step
namespace envar {
struct GNLayout {
  size_t D, Y, partial, tmp, G, grad, neg, Hc, info, total;
  int nsplit;
  long kchunk;
};

static GNLayout gn_layout(int n, long n_obs) {
  GNLayout L{};
  gram_split(n, n_obs, 8, L.nsplit, L.kchunk);
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t a = o;
    o = align256(o + b);
    return a;
  };
  L.D = take((size_t)(n + 1) * n_obs * 8);
  L.Y = take((size_t)n * n_obs * 8);
  L.partial = take((size_t)L.nsplit * n * n * 8);
  L.tmp = take((size_t)gram_reduce_groups(L.nsplit) * n * n * 8);
  L.G = take((size_t)n * n * 8);
  L.grad = take((size_t)n * 8);
  L.neg = take((size_t)n * 8);
  L.Hc = take((size_t)n * n * 8);
  L.info = take(256);
  L.total = o;
  return L;
}
}  // namespace envar

extern "C" size_t envar_gn_bytes(int32_t n, int64_t K) {
  if (n < 1 || K < 1) return 0;
  return gn_layout(n, (long)K * OBS_CHANNELS).total;
}

namespace envar {
// Gauss-Newton step on the device; the gradient stays in the workspace at L.grad
static int gn_step_impl(const double* series_dev, int n, long K, double eps, const double* w_dev, void* ws,
                        double* dw_dev, double* hgn_dev, double* jw_dev, hipStream_t s) {
  const long n_obs = K * OBS_CHANNELS;
  const GNLayout L = gn_layout(n, n_obs);
  double* D = at<double>(ws, L.D);
  double* Y = at<double>(ws, L.Y);
  double* G = at<double>(ws, L.G);
  double* grad = at<double>(ws, L.grad);
  const double shift = (double)(n - 1);  // (N_ens - 1) with N_ens = n members
  launch_obs_fluct(series_dev, n + 1, OBS_CHANNELS, (long)K, D, s);
  launch_yrows(D, n, n_obs, eps, Y, s);
  launch_gram<double>(Y, n, n_obs, n_obs, at<double>(ws, L.partial), L.nsplit, L.kchunk, s);
  launch_gram_reduce(at<double>(ws, L.partial), n, L.nsplit, at<double>(ws, L.tmp), G, s);
  launch_rowdot(Y, D, n, n_obs, 1.0, w_dev, shift, grad, s);  // Y^T d_0 + (N - 1) w
  launch_rowdot(D, D, 1, n_obs, 0.5, nullptr, 0.0, jw_dev, s);  // 1/2 |d_0|^2
  launch_rowdot(w_dev, w_dev, 1, n, 0.5 * shift, nullptr, 0.0, jw_dev + 1, s);  // 1/2 (N - 1) |w|^2
  launch_shift_diag(G, n, shift, hgn_dev, grad, at<double>(ws, L.neg), s);
  HIP_OK(hipMemcpyAsync(at<double>(ws, L.Hc), hgn_dev, (size_t)n * n * 8, hipMemcpyDeviceToDevice, s));
  if (launch_chol_solve(at<double>(ws, L.Hc), at<double>(ws, L.neg), n, dw_dev, at<double>(ws, L.info), s, 0.0))
    return fail(ENVAR_EDEVICE, "Cholesky launch failed (n = %d)", n);
  HIP_OK(hipGetLastError());
  return ENVAR_OK;
}
}  // namespace envar

extern "C" int envar_gn_step(const double* series_dev, int32_t n, int64_t K, double eps, const double* w_dev,
                             void* ws_dev, size_t ws_bytes, double* dw_dev, double* hgn_dev, double* jw_dev,
                             void* stream) {
  if (n < 1 || K < 1) return fail(ENVAR_EINVAL, "n and K must be >= 1");
  if (n > 1024) return fail(ENVAR_EINVAL, "n = %d exceeds 1024", n);
  if (!(eps > 0.0)) return fail(ENVAR_EINVAL, "eps must be positive");
  if (!series_dev || !w_dev || !ws_dev || !dw_dev || !hgn_dev || !jw_dev) return fail(ENVAR_EINVAL, "NULL device pointer");
  const GNLayout L = gn_layout(n, (long)K * OBS_CHANNELS);
  if (ws_bytes < L.total) return fail(ENVAR_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
  return gn_step_impl(series_dev, n, (long)K, eps, w_dev, ws_dev, dw_dev, hgn_dev, jw_dev, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------- EnVar loop over w
namespace envar {
struct EnsLayout {
  size_t rows, series, J, fws, gws, w, dw, H, jw, wt, jt, total;
  size_t fws_bytes, gws_bytes;
  long K;
};
static EnsLayout ens_layout(const Plan& P, int n, long m, int horizon, int every) {
  EnsLayout L{};
  L.K = horizon / every;
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t a = o;
    o = align256(o + b);
    return a;
  };
  L.rows = take((size_t)(n + 1) * m * 8);
  L.series = take((size_t)(n + 1) * OBS_CHANNELS * L.K * 8);
  L.J = take((size_t)(n + 1) * 8);
  L.fws_bytes = make_ws(P, n + 1).total;
  L.fws = take(L.fws_bytes);
  L.gws_bytes = gn_layout(n, L.K * OBS_CHANNELS).total;
  L.gws = take(L.gws_bytes);
  L.w = take((size_t)n * 8);
  L.dw = take((size_t)n * 8);
  L.H = take((size_t)n * n * 8);
  L.jw = take(2 * 8);
  L.wt = take((size_t)(n + 1) * n * 8);
  L.jt = take((size_t)(n + 1) * 8);
  L.total = o;
  return L;
}

// -H^-1 g by the two-loop recursion over the stored pairs (oldest first), initial scaling s.y / y.y
static std::vector<double> lbfgs_dir(const std::vector<double>& g, const std::deque<std::vector<double>>& S,
                                     const std::deque<std::vector<double>>& Yh) {
  const size_t n = g.size(), k = S.size();
  auto dot = [&](const std::vector<double>& a, const std::vector<double>& b) {
    double t = 0.0;
    for (size_t i = 0; i < n; ++i) t += a[i] * b[i];
    return t;
  };
  std::vector<double> q = g, alpha(k), rho(k);
  for (size_t kk = k; kk-- > 0;) {
    rho[kk] = 1.0 / dot(Yh[kk], S[kk]);
    alpha[kk] = rho[kk] * dot(S[kk], q);
    for (size_t i = 0; i < n; ++i) q[i] -= alpha[kk] * Yh[kk][i];
  }
  const double gamma = k ? dot(S[k - 1], Yh[k - 1]) / dot(Yh[k - 1], Yh[k - 1]) : 1.0;
  for (size_t i = 0; i < n; ++i) q[i] *= gamma;
  for (size_t kk = 0; kk < k; ++kk) {
    const double b = rho[kk] * dot(Yh[kk], q);
    for (size_t i = 0; i < n; ++i) q[i] += (alpha[kk] - b) * S[kk][i];
  }
  for (size_t i = 0; i < n; ++i) q[i] = -q[i];
  return q;
}
}  // namespace envar

extern "C" size_t envar_ens_bytes(const envar_problem* p, int32_t n, int64_t m, int32_t horizon, int32_t every) {
  Plan P;
  if (make_plan(p, P) != ENVAR_OK || n < 1 || m != P.m || horizon < 1) return 0;
  if (every < 1) every = 1;
  if (horizon / every < 1) return 0;
  return ens_layout(P, n, (long)m, horizon, every).total;
}

extern "C" int envar_ens_iterate(const envar_problem* p, const void* state_dev, const double* fe_dev,
                                 const double* E_dev, int32_t n, int64_t m, int32_t horizon,
                                 const envar_ens_params* prm_in, double* w_dev, void* ws_dev, size_t ws_bytes,
                                 envar_ens_record* recs, void* stream) {
  Plan P;
  int rc = make_plan(p, P);
  if (rc) return rc;
  if (!state_dev || !fe_dev || !E_dev || !w_dev || !ws_dev || !prm_in) return fail(ENVAR_EINVAL, "NULL pointer");
  if (n < 1 || n > 1024) return fail(ENVAR_EINVAL, "n must be in [1, 1024]");
  if (m != P.m) return fail(ENVAR_EINVAL, "m = %lld but the control region has m = %ld", (long long)m, P.m);
  if (horizon < 1) return fail(ENVAR_EINVAL, "horizon must be >= 1");
  if (!P.obs_ok) return fail(ENVAR_EINVAL, "the lid sensors need the cavity geometry");
  envar_ens_params prm = *prm_in;
  if (prm.method != ENVAR_GN && prm.method != ENVAR_LBFGS) return fail(ENVAR_EINVAL, "unknown method %d", prm.method);
  if (prm.iters < 1) return fail(ENVAR_EINVAL, "iters must be >= 1");
  if (prm.memory <= 0) prm.memory = 5;
  if (prm.max_trials <= 0) prm.max_trials = 10;
  if (!(prm.eps > 0.0)) prm.eps = 1e-4;
  if (!(prm.c1 > 0.0)) prm.c1 = 1e-4;
  if (!(prm.shrink > 0.0) || prm.shrink >= 1.0) prm.shrink = 0.5;
  if (prm.every <= 0) prm.every = 1;
  if (prm.trial_batch <= 0) prm.trial_batch = 8;
  if (horizon / prm.every < 1) return fail(ENVAR_EINVAL, "every must be in [1, horizon]");
  const EnsLayout L = ens_layout(P, n, (long)m, horizon, prm.every);
  if (ws_bytes < L.total) return fail(ENVAR_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
  hipStream_t s = (hipStream_t)stream;
  void* ws = ws_dev;
  double* rows = at<double>(ws, L.rows);
  double* series = at<double>(ws, L.series);
  double* wd = at<double>(ws, L.w);
  const size_t nb = (size_t)n * 8;
  std::vector<double> w(n), g(n), dw(n), jw(2), gprev, wprev;
  HIP_OK(hipMemcpyAsync(w.data(), w_dev, nb, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  std::deque<std::vector<double>> S, Yh;
  const double shift = (double)(n - 1);
  auto wdot = [&](const std::vector<double>& a) {
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += a[i] * a[i];
    return t;
  };
  // J(w_t) of several trial weights W [nt][n] in one batched forward (rows independent)
  std::vector<double> jt(n + 1);
  auto J_trials = [&](const std::vector<double>& W, int nt) -> int {
    HIP_OK(hipMemcpyAsync(at<double>(ws, L.wt), W.data(), (size_t)nt * nb, hipMemcpyHostToDevice, s));
    launch_combine_rows(fe_dev, E_dev, n, (long)m, at<double>(ws, L.wt), nt, rows, s);
    int r = forward_impl(P, state_dev, rows, nt, horizon, at<double>(ws, L.fws), L.fws_bytes, at<double>(ws, L.J),
                         nullptr, nullptr, s, false, series, prm.every);
    if (r) return r;
    double* D = at<double>(ws, L.gws);  // the step's fluctuation buffer, reused
    launch_obs_fluct(series, nt, OBS_CHANNELS, L.K, D, s);
    launch_rowdot(D, D, nt, L.K * OBS_CHANNELS, 0.5, nullptr, 0.0, at<double>(ws, L.jt), s, true);  // 1/2 |d_t|^2
    HIP_OK(hipMemcpyAsync(jt.data(), at<double>(ws, L.jt), (size_t)nt * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return ENVAR_OK;
  };
  for (int it = 0; it < prm.iters; ++it) {
    HIP_OK(hipMemcpyAsync(wd, w.data(), nb, hipMemcpyHostToDevice, s));
    launch_build_rows(fe_dev, E_dev, n, (long)m, wd, prm.eps, n + 1, rows, s);
    rc = forward_impl(P, state_dev, rows, n + 1, horizon, at<double>(ws, L.fws), L.fws_bytes, at<double>(ws, L.J),
                      nullptr, nullptr, s, false, series, prm.every);
    if (rc) return rc;
    rc = gn_step_impl(series, n, L.K, prm.eps, wd, at<double>(ws, L.gws), at<double>(ws, L.dw),
                      at<double>(ws, L.H), at<double>(ws, L.jw), s);
    if (rc) return rc;
    const GNLayout GL = gn_layout(n, L.K * OBS_CHANNELS);
    HIP_OK(hipMemcpyAsync(g.data(), at<double>(at<char>(ws, L.gws), GL.grad), nb, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(dw.data(), at<double>(ws, L.dw), nb, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(jw.data(), at<double>(ws, L.jw), 2 * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i)
      if (!std::isfinite(g[i])) return fail(ENVAR_EDIVERGED, "non-finite gradient at iteration %d", it);
    if (!gprev.empty()) {
      std::vector<double> sv(n), yv(n);
      double sy = 0.0;
      for (int i = 0; i < n; ++i) {
        sv[i] = w[i] - wprev[i];
        yv[i] = g[i] - gprev[i];
        sy += sv[i] * yv[i];
      }
      if (sy > 0.0) {
        S.push_back(sv);
        Yh.push_back(yv);
        if ((int)S.size() > prm.memory) {
          S.pop_front();
          Yh.pop_front();
        }
      }
    }
    const double J = jw[0] + jw[1];
    double alpha = 1.0;
    int trials = 0, trial_rows = 0;
    std::vector<double> step(n, 0.0);
    if (prm.method == ENVAR_GN) {
      step = dw;
    } else {
      const std::vector<double> d = lbfgs_dir(g, S, Yh);
      double gd = 0.0;
      for (int i = 0; i < n; ++i) gd += g[i] * d[i];
      bool ok = false;
      // the trial steps 1, shrink, shrink^2, ... are evaluated trial_batch at a time; the first
      // one meeting the Armijo condition is taken, as a one-at-a-time search would
      const int B = std::min(prm.trial_batch, n + 1);
      double a = 1.0;
      while (trials < prm.max_trials && !ok) {
        const int nt = std::min(B, prm.max_trials - trials);
        std::vector<double> W((size_t)nt * n), at_(nt);
        for (int t = 0; t < nt; ++t) {
          at_[t] = a;
          for (int i = 0; i < n; ++i) W[(size_t)t * n + i] = w[i] + a * d[i];
          a *= prm.shrink;
        }
        rc = J_trials(W, nt);
        if (rc) return rc;
        trial_rows += nt;
        for (int t = 0; t < nt && !ok; ++t) {
          ++trials;
          double p2 = 0.0;
          for (int i = 0; i < n; ++i) p2 += W[(size_t)t * n + i] * W[(size_t)t * n + i];
          const double Jt = jt[t] + 0.5 * shift * p2;
          if (Jt <= J + prm.c1 * at_[t] * gd) {
            ok = true;
            alpha = at_[t];
            for (int i = 0; i < n; ++i) step[i] = alpha * d[i];
          }
        }
      }
      if (!ok) alpha = 0.0;
    }
    if (recs) {
      recs[it].J = J;
      recs[it].J_obs = jw[0];
      recs[it].J_prior = jw[1];
      recs[it].gnorm = std::sqrt(wdot(g));
      recs[it].alpha = alpha;
      recs[it].trials = trials;
      recs[it].trial_rows = trial_rows;
    }
    gprev = g;
    wprev = w;
    for (int i = 0; i < n; ++i) w[i] += step[i];
    if (prm.method == ENVAR_LBFGS && alpha == 0.0) {
      for (int k = it + 1; k < prm.iters && recs; ++k) recs[k] = envar_ens_record{NAN, NAN, NAN, NAN, 0.0, 0, 0};  // not run
      break;
    }
  }
  HIP_OK(hipMemcpyAsync(w_dev, w.data(), nb, hipMemcpyHostToDevice, s));
  HIP_OK(hipStreamSynchronize(s));
  return ENVAR_OK;
}

// ---------------------------------------------------------------------------- eigen-ensemble
namespace envar {
struct EigSetup {
  envar_eigen_params prm;
  int i0, j0, nxb, nyb, ncc, npos, N, b;
  long M;
  std::vector<int> bidx;  // rectangle index of each control cell, in control order
};

static int eig_setup(const Plan& P, int N, const envar_eigen_params* in, EigSetup& S) {
  envar_eigen_params prm{};
  if (in) prm = *in;
  if (!(prm.a_x > 0.0)) prm.a_x = 0.07;
  if (!(prm.a_y > 0.0)) prm.a_y = 0.07;
  if (!(prm.sigma2_max > 0.0)) prm.sigma2_max = 0.01;
  if (!(prm.tol > 0.0)) prm.tol = 1e-10;
  if (prm.max_iters <= 0) prm.max_iters = 500;
  if (prm.taper != ENVAR_TAPER_NONE && prm.taper != ENVAR_TAPER_ELLIPSE)
    return fail(ENVAR_EINVAL, "unknown taper %d", prm.taper);
  if (prm.component != 0 && prm.component != 1) return fail(ENVAR_EINVAL, "component must be 0 (x) or 1 (y)");
  if (N < 2 || N > 448) return fail(ENVAR_EINVAL, "N = %d must be in [2, 448]", N);
  const Geo& g = P.lev[0];
  int imin = 1 << 30, imax = -1, jmin = 1 << 30, jmax = -1;
  for (int c : P.ctrl_cells) {
    const int i = c % g.nx, j = c / g.nx;
    imin = std::min(imin, i);
    imax = std::max(imax, i);
    jmin = std::min(jmin, j);
    jmax = std::max(jmax, j);
  }
  S.ncc = (int)P.ctrl_cells.size();
  if (S.ncc < 2) return fail(ENVAR_EINVAL, "the control region has %d cell(s)", S.ncc);
  S.i0 = imin;
  S.j0 = jmin;
  S.nxb = imax - imin + 1;
  S.nyb = jmax - jmin + 1;
  S.M = (long)S.nxb * S.nyb;
  S.bidx.resize(S.ncc);
  S.npos = 0;
  for (int k = 0; k < S.ncc; ++k) {
    const int i = P.ctrl_cells[k] % g.nx - imin, j = P.ctrl_cells[k] / g.nx - jmin;
    S.bidx[k] = j * S.nxb + i;
    bool pos = true;
    if (prm.taper == ENVAR_TAPER_ELLIPSE) {  // the same test as the device's taper
      const double ex = ((i + 0.5) * g.h - 0.5 * S.nxb * g.h) / (0.5 * S.nxb * g.h);
      const double ey = ((j + 0.5) * g.h - 0.5 * S.nyb * g.h) / (0.5 * S.nyb * g.h);
      pos = ex * ex + ey * ey < 1.0;
    }
    S.npos += pos;
  }
  if (N > S.npos) return fail(ENVAR_EINVAL, "N = %d exceeds the %d control cells with sigma > 0", N, S.npos);
  if (prm.oversample <= 0) prm.oversample = std::max(8, N / 2);
  S.b = std::min(std::min(N + prm.oversample, 512), S.npos);
  S.N = N;
  S.prm = prm;
  return ENVAR_OK;
}

struct EigLayout {
  size_t sig, Kx, Ky, bidx, QZ, W1, T1, UV, partial, tmp, G2, Ts, ZZ, QQ, Wm, Wt, M1, Pm, Gy, Pg, Pgt, Sm, Cm, theta,
      lam, ninv, dv, resid, jac, total;
  int nsplit;
  long kchunk;
};

static EigLayout eig_layout(const EigSetup& S) {
  EigLayout L{};
  const int b = S.b, n2 = 2 * b;
  gram_split(n2, S.M, 8, L.nsplit, L.kchunk);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t a = o;
    o = align256(o + bytes);
    return a;
  };
  const size_t bb = (size_t)b * b * 8, bm = (size_t)b * S.M * 8;
  L.sig = take((size_t)S.M * 8);
  L.Kx = take((size_t)S.nxb * S.nxb * 8);
  L.Ky = take((size_t)S.nyb * S.nyb * 8);
  L.bidx = take((size_t)S.ncc * 4);
  L.QZ = take(2 * bm);
  L.W1 = take(bm);
  L.T1 = take(bm);
  L.UV = take(2 * bm);
  L.partial = take((size_t)L.nsplit * n2 * n2 * 8);
  L.tmp = take((size_t)gram_reduce_groups(L.nsplit) * n2 * n2 * 8);
  L.G2 = take((size_t)n2 * n2 * 8);
  L.Ts = take(bb);
  L.ZZ = take(bb);
  L.QQ = take(bb);
  L.Wm = take(bb);
  L.Wt = take(bb);
  L.M1 = take(bb);
  L.Pm = take(bb);
  L.Gy = take(bb);
  L.Pg = take(bb);
  L.Pgt = take(bb);
  L.Sm = take(bb);
  L.Cm = take(bb);
  L.theta = take((size_t)b * 8);
  L.lam = take((size_t)b * 8);
  L.ninv = take((size_t)b * 8);
  L.dv = take((size_t)b * 8);
  L.resid = take((size_t)b * eig_resid_split() * 8);
  L.jac = take(std::max<size_t>(8, jacobi_scratch_doubles(b) * 8));
  L.total = o;
  return L;
}
}  // namespace envar

extern "C" size_t envar_eigen_bytes(const envar_problem* p, int32_t N, const envar_eigen_params* params) {
  Plan P;
  if (make_plan(p, P) != ENVAR_OK) return 0;
  EigSetup S;
  if (eig_setup(P, N, params, S) != ENVAR_OK) return 0;
  return eig_layout(S).total;
}

extern "C" int envar_eigen_ensemble(const envar_problem* p, int32_t N, const envar_eigen_params* params,
                                    double* E_dev, double* mu_dev, void* ws_dev, size_t ws_bytes,
                                    envar_eigen_info* info, void* stream) {
  Plan P;
  int rc = make_plan(p, P);
  if (rc) return rc;
  EigSetup S;
  rc = eig_setup(P, N, params, S);
  if (rc) return rc;
  if (!E_dev || !mu_dev || !ws_dev) return fail(ENVAR_EINVAL, "NULL device pointer");
  const EigLayout L = eig_layout(S);
  if (ws_bytes < L.total) return fail(ENVAR_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
  hipStream_t s = (hipStream_t)stream;
  void* ws = ws_dev;
  const int b = S.b;
  const long M = S.M;
  const double h = P.lev[0].h;
  double* sig = at<double>(ws, L.sig);
  double* Kx = at<double>(ws, L.Kx);
  double* Ky = at<double>(ws, L.Ky);
  int* bidx = at<int>(ws, L.bidx);
  double* Q = at<double>(ws, L.QZ);
  double* Z = Q + (size_t)b * M;
  double* W1 = at<double>(ws, L.W1);
  double* T1 = at<double>(ws, L.T1);
  double* U = at<double>(ws, L.UV);
  double* Vv = U + (size_t)b * M;
  double* G2 = at<double>(ws, L.G2);
  auto d = [&](size_t off) { return at<double>(ws, off); };
  HIP_OK(hipMemcpyAsync(bidx, S.bidx.data(), (size_t)S.ncc * 4, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemsetAsync(sig, 0, (size_t)M * 8, s));
  launch_eig_sigma(bidx, S.ncc, S.nxb, S.nyb, h, S.prm.sigma2_max, S.prm.taper, sig, s);
  launch_kernel1d(S.nxb, h, S.prm.a_x, Kx, s);
  launch_kernel1d(S.nyb, h, S.prm.a_y, Ky, s);
  // Z = B Q = D (Ky kron Kx) D Q, rows of Q as ny x nx grids
  auto apply_B = [&]() {
    launch_scale_rows(Q, sig, b, M, W1, s);
    launch_dgemm(b * S.nyb, S.nxb, S.nxb, W1, S.nxb, 0, Kx, S.nxb, 0, T1, S.nxb, 0, 1, nullptr, 0, s);
    launch_dgemm(S.nyb, S.nxb, S.nyb, Ky, S.nyb, 0, T1, S.nxb, M, Z, S.nxb, M, b, sig, S.nxb, s);
  };
  auto gram2 = [&](int rows) {  // G2 = X X^T over the first `rows` rows of [Q; Z]
    launch_gram<double>(Q, rows, M, M, d(L.partial), L.nsplit, L.kchunk, s);
    launch_gram_reduce(d(L.partial), rows, L.nsplit, d(L.tmp), G2, s);
  };
  // One Jacobi sweep per iteration: the next block spans B Q whatever rotation W the Ritz step
  // applies, so the subspace iteration is unchanged; the basis carries the rotations over from one
  // iteration to the next, and the residual test (every kept |B u - theta u| from the rotated
  // blocks) only passes once that basis diagonalises the Ritz matrix. Measured at h = 1/128: the
  // same iteration counts (69 for 20 members, 39 for 64) and eigenvalues within 1e-15 relative as
  // with sweeps until convergence, in 15 against 20 ms and 41 against 78 ms.
  auto jacobi = [&](const double* A, double* ev, double* Wc, double* Wr) -> int {
    if (launch_jacobi(A, b, b, ev, Wc, Wr, d(L.jac), s, 1)) return fail(ENVAR_EDEVICE, "Jacobi launch failed");
    return ENVAR_OK;
  };
  auto chol_inv = [&](const double* G, double* Li) -> int {
    if (launch_chol_inv(G, b, Li, d(L.jac), s)) return fail(ENVAR_EDEVICE, "Cholesky launch failed");
    return ENVAR_OK;
  };
  // start block: random on the cells with sigma > 0, orthonormalised: Q = L^-1 Q0 with L L^T = Q0 Q0^T
  launch_eig_random(Z, b, M, sig, S.prm.seed ? S.prm.seed : 0x5EEDull, s);
  launch_gram<double>(Z, b, M, M, d(L.partial), L.nsplit, L.kchunk, s);
  launch_gram_reduce(d(L.partial), b, L.nsplit, d(L.tmp), d(L.Gy), s);
  if ((rc = chol_inv(d(L.Gy), d(L.Sm)))) return rc;
  launch_dgemm(b, (int)M, b, d(L.Sm), b, 0, Z, M, 0, Q, M, 0, 1, nullptr, 0, s);
  HIP_OK(hipGetLastError());
  const int rsplit = eig_resid_split();
  // the Ritz values and residual partials come back every iteration for the convergence test:
  // through one pinned buffer of this host thread (kept for the process), not pageable memory
  static thread_local double* pin = nullptr;
  static thread_local size_t pin_n = 0;
  const size_t need = (size_t)b + (size_t)S.N * rsplit;
  if (pin_n < need) {
    if (pin) (void)hipHostFree(pin);
    pin = nullptr;
    pin_n = 0;
    HIP_OK(hipHostMalloc((void**)&pin, need * sizeof(double), hipHostMallocDefault));
    pin_n = need;
  }
  const double* const th = pin;
  const double* const res = pin + b;
  int it = 0;
  bool conv = false;
  double maxr = 0.0;
  for (it = 1; it <= S.prm.max_iters; ++it) {
    apply_B();
    gram2(2 * b);
    launch_eig_blocks(G2, b, d(L.Ts), d(L.ZZ), d(L.QQ), s);
    if ((rc = jacobi(d(L.Ts), d(L.theta), d(L.Wm), d(L.Wt)))) return rc;
    // Ritz vectors and images: [U; V] = W^T [Q; Z]
    launch_dgemm(b, (int)M, b, d(L.Wt), b, 0, Q, M, (long)b * M, U, M, (long)b * M, 2, nullptr, 0, s);
    launch_eig_resid(U, Vv, d(L.theta), S.N, M, d(L.resid), s);
    HIP_OK(hipMemcpyAsync(pin, d(L.theta), (size_t)b * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(pin + b, d(L.resid), (size_t)S.N * rsplit * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    maxr = 0.0;
    for (int k = 0; k < S.N; ++k) {
      double r2 = 0.0;
      for (int q = 0; q < rsplit; ++q) r2 += res[(size_t)k * rsplit + q];
      maxr = std::max(maxr, std::sqrt(r2));
    }
    maxr = th[0] > 0.0 ? maxr / th[0] : INFINITY;
    if (!std::isfinite(maxr)) return fail(ENVAR_EDIVERGED, "non-finite Ritz values at iteration %d", it);
    if (maxr <= S.prm.tol) {
      conv = true;
      break;
    }
    if (it == S.prm.max_iters) break;
    // next Q: Cholesky orthonormalisation of the unit-norm rows of V = W^T Z (in decreasing Ritz
    // value), Q = L^-1 Dn^-1 W^T Z with P = W^T (Z Z^T) W, Dn = diag(P)^1/2, L L^T = Dn^-1 P Dn^-1
    launch_small_gemm(b, d(L.ZZ), 0, d(L.Wm), 0, nullptr, d(L.M1), s);
    launch_small_gemm(b, d(L.Wt), 0, d(L.M1), 0, nullptr, d(L.Pm), s);
    launch_eig_unit_gram(d(L.Pm), b, d(L.Gy), d(L.ninv), s);
    if ((rc = chol_inv(d(L.Gy), d(L.Sm)))) return rc;
    launch_small_gemm(b, d(L.Sm), 0, d(L.Wt), 0, d(L.ninv), d(L.Cm), s);
    launch_dgemm(b, (int)M, b, d(L.Cm), b, 0, Z, M, 0, Q, M, 0, 1, nullptr, 0, s);
    HIP_OK(hipGetLastError());
  }
  launch_eig_extract(U, d(L.theta), S.N, M, bidx, S.ncc, S.prm.component, E_dev, mu_dev, s);
  HIP_OK(hipGetLastError());
  if (info) {
    // orthonormality of the kept Ritz vectors: W^T (Q Q^T) W
    launch_small_gemm(b, d(L.QQ), 0, d(L.Wm), 0, nullptr, d(L.M1), s);
    launch_small_gemm(b, d(L.Wt), 0, d(L.M1), 0, nullptr, d(L.Pm), s);
    std::vector<double> pm((size_t)b * b);
    HIP_OK(hipMemcpyAsync(pm.data(), d(L.Pm), pm.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    double oe = 0.0;
    for (int i = 0; i < S.N; ++i)
      for (int j = 0; j < S.N; ++j) oe = std::max(oe, std::fabs(pm[(size_t)i * b + j] - (i == j ? 1.0 : 0.0)));
    info->iters = std::min(it, S.prm.max_iters);
    info->converged = conv;
    info->block = b;
    info->reserved = 0;
    info->max_resid = maxr;
    info->orth_err = oe;
  }
  HIP_OK(hipStreamSynchronize(s));
  return ENVAR_OK;
}

extern "C" size_t envar_recon_bytes(int32_t N, int64_t m) {
  if (N < 1 || m < 1) return 0;
  return align256((size_t)N * 8) * 3 + align256((size_t)recon_blocks(m) * 16);
}

extern "C" int envar_recon_error(const double* E_dev, int32_t N, int64_t m, const double* f_dev, void* ws_dev,
                                 size_t ws_bytes, double* out_dev, void* stream) {
  if (N < 1 || m < 1) return fail(ENVAR_EINVAL, "N and m must be >= 1");
  if (!E_dev || !f_dev || !ws_dev || !out_dev) return fail(ENVAR_EINVAL, "NULL device pointer");
  const size_t need = envar_recon_bytes(N, m);
  if (ws_bytes < need) return fail(ENVAR_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  const size_t a = align256((size_t)N * 8);
  double* ef = at<double>(ws_dev, 0);
  double* ee = at<double>(ws_dev, a);
  double* coef = at<double>(ws_dev, 2 * a);
  double* part = at<double>(ws_dev, 3 * a);
  launch_rowdot(E_dev, f_dev, N, (long)m, 1.0, nullptr, 0.0, ef, s);
  launch_rowdot(E_dev, E_dev, N, (long)m, 1.0, nullptr, 0.0, ee, s, true);
  launch_recon(E_dev, N, (long)m, f_dev, ef, ee, coef, part, out_dev, s);
  HIP_OK(hipGetLastError());
  return ENVAR_OK;
}

extern "C" size_t envar_posterior_bytes(int32_t n) {
  if (n < 1) return 0;
  return align256((size_t)n * n * 8) + 256;
}

extern "C" int envar_posterior_var(const double* controls_dev, int32_t n, int64_t m, double eps, const double* hgn_dev,
                                   void* ws_dev, size_t ws_bytes, double* var_dev, void* stream) {
  if (n < 1 || m < 1) return fail(ENVAR_EINVAL, "n and m must be >= 1");
  if (n > 128) return fail(ENVAR_EINVAL, "n = %d exceeds 128", n);
  if (!(eps > 0.0)) return fail(ENVAR_EINVAL, "eps must be positive");
  if (!controls_dev || !hgn_dev || !ws_dev || !var_dev) return fail(ENVAR_EINVAL, "NULL device pointer");
  if (ws_bytes < envar_posterior_bytes(n)) return fail(ENVAR_ENOMEM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  double* C = (double*)ws_dev;
  double* info = at<double>(ws_dev, align256((size_t)n * n * 8));
  launch_spd_inverse(hgn_dev, n, C, info, s);
  if (launch_post_var(controls_dev, n, (long)m, eps, C, var_dev, s))
    return fail(ENVAR_EDEVICE, "posterior variance launch failed (n = %d)", n);
  HIP_OK(hipGetLastError());
  return ENVAR_OK;
}

// ---------------------------------------------------------------------------- iterate
namespace envar {
struct IterLayout {
  size_t rows, J, g, fwd, grad, total;
};
static IterLayout iter_layout(const Plan& P, int n) {
  IterLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t a = o;
    o = align256(o + b);
    return a;
  };
  L.rows = take((size_t)(n + 1) * P.m * 8);
  L.J = take((size_t)(n + 1) * 8);
  L.g = take((size_t)P.m * 8);
  L.fwd = take(make_ws(P, n + 1).total);
  L.grad = take(grad_layout(n, P.m, P.p.precision).total);
  L.total = o;
  return L;
}

__global__ void k_rows(const double* f, const double* pert, int n, long m, double* rows, double alpha,
                       const double* g, double* ftrial);
}  // namespace envar

extern "C" size_t envar_iterate_bytes(const envar_problem* p, int32_t n, int64_t m) {
  Plan P;
  if (make_plan(p, P) || n < 1 || m != P.m) return 0;
  return iter_layout(P, n).total;
}

namespace envar {
__global__ void k_rows(const double* f, const double* pert, int n, long m, double* rows, double alpha,
                       const double* g, double* ftrial) {
  // rows[0] = f, rows[i] = f + pert[i-1]; ftrial = f - alpha g (when g != NULL)
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < m; k += (long)gridDim.x * blockDim.x) {
    const double fk = f[k];
    if (rows) {
      rows[k] = fk;
      for (int i = 0; i < n; ++i) rows[(long)(i + 1) * m + k] = fk + pert[(long)i * m + k];
    }
    if (g) ftrial[k] = fk - alpha * g[k];
  }
}

}  // namespace envar

extern "C" int envar_iterate(const envar_problem* p, const void* state_dev, double* f_dev, const double* perturb_dev, int32_t n,
                  int64_t m, int32_t horizon, const envar_ls_params* ls, void* ws_dev, size_t ws_bytes,
                  envar_iter_record* records, void* stream) {
  Plan P;
  int rc = make_plan(p, P);
  if (rc) return rc;
  if (!ls || ls->iters < 1) return fail(ENVAR_EINVAL, "ls->iters must be >= 1");
  if (m != P.m || n < 1) return fail(ENVAR_EINVAL, "bad n or m");
  if (!state_dev || !f_dev || !perturb_dev || !ws_dev) return fail(ENVAR_EINVAL, "NULL device pointer");
  const IterLayout L = iter_layout(P, n);
  if (ws_bytes < L.total) return fail(ENVAR_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
  hipStream_t s = (hipStream_t)stream;
  const int trials = ls->max_trials > 0 ? ls->max_trials : 8;
  const double c1 = ls->c1 > 0 ? ls->c1 : 1e-4, shrink = ls->shrink > 0 ? ls->shrink : 0.5;
  double* rows = at<double>(ws_dev, L.rows);
  double* Jd = at<double>(ws_dev, L.J);
  double* g = at<double>(ws_dev, L.g);
  void* fws = at<char>(ws_dev, L.fwd);
  void* gws = at<char>(ws_dev, L.grad);
  const size_t fbytes = make_ws(P, n + 1).total;
  const size_t gbytes = grad_layout(n, P.m, P.p.precision).total;
  // max |perturb| for the default first step
  std::vector<double> hp((size_t)n * m), hg(m);
  HIP_OK(hipMemcpyAsync(hp.data(), perturb_dev, hp.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  double pmax = 0.0;
  for (double x : hp) pmax = std::max(pmax, std::fabs(x));
  double alpha_fixed = -1.0;
  const int grid = (int)std::min<long>(4096, (m + 255) / 256);
  for (int it = 0; it < ls->iters; ++it) {
    hipLaunchKernelGGL(k_rows, dim3(grid), dim3(256), 0, s, f_dev, perturb_dev, n, (long)m, rows, 0.0,
                       (const double*)nullptr, (double*)nullptr);
    rc = forward_impl(P, state_dev, rows, n + 1, horizon, fws, fbytes, Jd, nullptr, nullptr, s, false);
    if (rc) return rc;
    rc = envar_gradient(rows, Jd, n, m, P.p.precision, gws, gbytes, g, s);
    if (rc) return rc;
    double J0 = 0.0;
    HIP_OK(hipMemcpyAsync(&J0, Jd, 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(hg.data(), g, (size_t)m * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    double gg = 0.0, gmax = 0.0;
    for (double x : hg) {
      gg += x * x;
      gmax = std::max(gmax, std::fabs(x));
    }
    envar_iter_record rec{J0, std::sqrt(gg), 0.0, NAN};
    const bool search = alpha_fixed < 0.0 || (ls->search_every > 0 && it % ls->search_every == 0);
    double alpha = alpha_fixed;
    if (search) {
      double a = ls->alpha0 > 0 ? ls->alpha0 : pmax / std::max(gmax, 1e-300);
      bool ok = false;
      // Backtracking with the trial rows f - a g, a = a0, a0 shrink, ..., up to n + 1 of them per
      // batched forward (a forward of a few rows takes about as long as one: a single member
      // leaves most of the GPU idle). Each member's cost is that of its own forward, so the first
      // acceptable trial in order is the one that trying them one after another accepts.
      std::vector<double> Jt((size_t)n + 1);
      for (int t = 0; t < trials && !ok;) {
        const int nb = std::min(trials - t, n + 1);
        double at_ = a;
        for (int q = 0; q < nb; ++q, at_ *= shrink)
          hipLaunchKernelGGL(k_rows, dim3(grid), dim3(256), 0, s, f_dev, perturb_dev, 0, (long)m, (double*)nullptr,
                             at_, (const double*)g, rows + (long)q * m);
        rc = forward_impl(P, state_dev, rows, nb, horizon, fws, fbytes, Jd, nullptr, nullptr, s, false);
        if (rc) return rc;
        HIP_OK(hipMemcpyAsync(Jt.data(), Jd, (size_t)nb * 8, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        for (int q = 0; q < nb; ++q) {
          if (Jt[q] <= J0 - c1 * a * gg) {
            ok = true;
            rec.J_trial = Jt[q];
            break;
          }
          a *= shrink;
        }
        t += nb;
      }
      if (!ok) {
        if (records) records[it] = rec;
        return ENVAR_OK;
      }
      alpha = a;
      alpha_fixed = a;
    }
    rec.alpha = alpha;
    // f <- f - alpha g
    hipLaunchKernelGGL(k_rows, dim3(grid), dim3(256), 0, s, f_dev, perturb_dev, 0, (long)m, (double*)nullptr, alpha,
                       (const double*)g, f_dev);
    HIP_OK(hipGetLastError());
    if (records) records[it] = rec;
  }
  HIP_OK(hipStreamSynchronize(s));
  return ENVAR_OK;
}


// ============================================================================ serving
namespace envar {

// first-fit allocator over the caller's device pool (offsets only)
struct PoolAlloc {
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes
  void init(size_t n) {
    size = n & ~size_t(255);
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t n, size_t& off) {
    n = align256(n);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        off = it->first;
        const size_t rem = it->second - n;
        free_.erase(it);
        if (rem) free_[off + n] = rem;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align256(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct ReqLayout {
  size_t ws, ctrl, J, total;
};
static ReqLayout req_layout(const Plan& P, int n) {
  ReqLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t a = o;
    o = align256(o + b);
    return a;
  };
  L.ws = take(make_ws(P, n).total);
  L.ctrl = take((size_t)n * P.m * 8);
  L.J = take((size_t)n * 8);
  L.total = o;
  return L;
}

struct Request {
  uint64_t ticket = 0;
  int n = 0, horizon = 0;
  std::vector<double> controls;
  Plan P;
  ReqLayout L{};
  size_t off = 0;
  Job job;
  double* J_pinned = nullptr;  // host staging: J [n], then stats [n][STATS_STRIDE], then max |div| [n]
  hipEvent_t done_ev = nullptr;
  std::vector<double> J;
  envar_request_stats st{};
  int phase = 0;  // 0 queued, 1 running, 2 finishing, 3 done
};

struct Server {
  envar_server_config cfg{};
  char* pool = nullptr;
  PoolAlloc alloc;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> table;
  std::vector<Request*> running, finishing;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  hipStream_t s = nullptr;
  std::chrono::steady_clock::time_point t0;
  Driver D;
  std::string err;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  template <typename TT>
  void loop() {
    (void)hipSetDevice(device);
    D.cap_max = 0;
    for (;;) {
      std::vector<Request*> admitted;
      {
        std::unique_lock<std::mutex> lk(mu);
        if (stop) break;
        while (!queue.empty() && (int)running.size() < cfg.max_jobs) {
          Request* r = queue.front();
          size_t off;
          if (!alloc.alloc(r->L.total, off)) break;  // FIFO: wait for memory
          queue.pop_front();
          r->off = off;
          r->phase = 1;
          r->st.start_s = now();
          running.push_back(r);
          admitted.push_back(r);
        }
        if (running.empty() && finishing.empty()) {
          cv_work.wait(lk, [&] { return stop || !queue.empty(); });
          continue;
        }
      }
      bool dev_err = false;
      for (Request* r : admitted) {
        char* base = pool + r->off;
        const hipError_t e =
            hipMemcpyAsync(base + r->L.ctrl, r->controls.data(), r->controls.size() * 8, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
          device_error(r, "control upload", e);
          dev_err = true;
          break;
        }
        r->job.ws = base + r->L.ws;
        r->job.ctrl = (const double*)(base + r->L.ctrl);
        if (tune_job<TT>(r->job, s) != ENVAR_OK) apply_choice(r->job, TileChoice());
        init_members<TT>(r->job, s);
        D.cap_max = std::max(D.cap_max, r->P.cap_max);
        if (D.cap == 0) D.cap = D.cap_max;
        ++D.epoch;
      }
      if (dev_err) break;
      if (!running.empty()) {
        std::vector<Job*> jobs;
        int left = 1 << 30;
        for (Request* r : running) {
          jobs.push_back(&r->job);
          left = std::min(left, r->job.horizon - r->job.step);
          r->st.peak_jobs = std::max(r->st.peak_jobs, (int)running.size());
        }
        const int rc = D.step<TT>(jobs, s, nullptr, left, !(cfg.flags & ENVAR_FLAG_NO_GRAPHS));
        if (rc) {
          std::lock_guard<std::mutex> lk(mu);
          err = g_err;
          stop = true;
          cv_done.notify_all();
          break;
        }
        bool changed = false;
        for (size_t k = 0; k < running.size();) {
          Request* r = running[k];
          if (r->job.step >= r->job.horizon) {
            double* Jd = (double*)(pool + r->off + r->L.J);
            finish_job(r->job, Jd, nullptr, false, s);
            const size_t n = (size_t)r->n;
            hipError_t e = hipMemcpyAsync(r->J_pinned, Jd, n * 8, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
              e = hipMemcpyAsync(r->J_pinned + n, r->job.w_<double>(r->job.w.stats), n * STATS_STRIDE * 8,
                                 hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
              e = hipMemcpyAsync(r->J_pinned + n * (1 + STATS_STRIDE), r->job.w_<double>(r->job.w.divmax), n * 8,
                                 hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipEventRecord(r->done_ev, s);
            if (e != hipSuccess) {
              running.erase(running.begin() + k);
              device_error(r, "result download", e);
              dev_err = true;
              break;
            }
            r->phase = 2;
            finishing.push_back(r);
            running.erase(running.begin() + k);
            changed = true;
          } else {
            ++k;
          }
        }
        if (changed) ++D.epoch;
        if (dev_err) break;
      }
      // completions
      for (size_t k = 0; k < finishing.size();) {
        Request* r = finishing[k];
        hipError_t q = hipEventQuery(r->done_ev);
        if (q == hipErrorNotReady && running.empty()) q = hipEventSynchronize(r->done_ev);
        if (q != hipSuccess && q != hipErrorNotReady) {
          finishing.erase(finishing.begin() + k);
          device_error(r, "completion event", q);
          dev_err = true;
          break;
        }
        if (q == hipSuccess) {
          const size_t n = (size_t)r->n;
          r->J.assign(r->J_pinned, r->J_pinned + n);
          bool finite = true;
          for (double x : r->J) finite = finite && std::isfinite(x);
          double cyc = 0.0, steps = 0.0, unconv = 0.0, mdiv = 0.0;
          for (size_t i = 0; i < n; ++i) {
            const double* m = r->J_pinned + n + i * STATS_STRIDE;
            cyc += m[ST_CYCLES];
            steps += m[ST_STEPS];
            unconv += m[ST_UNCONV];
            const double d = r->J_pinned[n * (1 + STATS_STRIDE) + i];
            mdiv = (d > mdiv || d != d) ? d : mdiv;
          }
          std::lock_guard<std::mutex> lk(mu);
          r->st.done_s = now();
          r->st.latency_s = r->st.done_s - r->st.submit_s;
          r->st.queue_s = r->st.start_s - r->st.submit_s;
          r->st.max_div = mdiv;
          r->st.mean_cycles = steps > 0 ? cyc / steps : 0.0;
          r->st.unconverged = (int)unconv;
          r->st.status = !finite ? ENVAR_EDIVERGED : unconv > 0 ? ENVAR_EUNCONVERGED : ENVAR_OK;
          alloc.release(r->off, r->L.total);
          r->phase = 3;
          finishing.erase(finishing.begin() + k);
          cv_done.notify_all();
        } else {
          ++k;
        }
      }
      if (dev_err) break;
    }
    D.drain();
    (void)hipStreamSynchronize(s);
    // the stream is drained and is destroyed before the Driver: no graph may wait on it later
    D.G.destroy_drained();
  }

  // A HIP call of the worker failed: the request completes with ENVAR_EDEVICE and the
  // server stops (pending and running requests then complete as cancelled).
  void device_error(Request* r, const char* what, hipError_t e) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(mu);
    err = buf;
    r->st.status = ENVAR_EDEVICE;
    r->st.done_s = now();
    r->st.latency_s = r->st.done_s - r->st.submit_s;
    r->phase = 3;
    stop = true;
    cv_done.notify_all();
  }
};

}  // namespace envar

struct envar_server {
  envar::Server impl;
};

extern "C" {

size_t envar_request_bytes(const envar_problem* p, int32_t n_rows) {
  Plan P;
  if (make_plan(p, P) || n_rows < 1) return 0;
  return req_layout(P, n_rows).total;
}

int envar_server_create(const envar_server_config* cfg, void* pool_dev, size_t pool_bytes, envar_server** out) {
  if (!cfg || !pool_dev || !out) return fail(ENVAR_EINVAL, "cfg, pool_dev and out are required");
  if (cfg->max_jobs < 1 || cfg->max_jobs > MAX_SEG) return fail(ENVAR_EINVAL, "max_jobs must be in [1, %d]", MAX_SEG);
  if (cfg->precision != ENVAR_FP64 && cfg->precision != ENVAR_MIXED) return fail(ENVAR_EINVAL, "unknown precision");
  auto* srv = new envar_server;
  Server& S = srv->impl;
  S.cfg = *cfg;
  if (S.cfg.max_queue <= 0) S.cfg.max_queue = 1024;
  S.pool = (char*)pool_dev;
  S.alloc.init(pool_bytes);
  S.t0 = std::chrono::steady_clock::now();
  if (hipGetDevice(&S.device) != hipSuccess || hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking) != hipSuccess) {
    delete srv;
    return fail(ENVAR_EDEVICE, "cannot create the server stream");
  }
  if (S.cfg.precision == ENVAR_MIXED)
    S.worker = std::thread([&S] { S.loop<float>(); });
  else
    S.worker = std::thread([&S] { S.loop<double>(); });
  *out = srv;
  return ENVAR_OK;
}

int envar_submit(envar_server* srv, const envar_request* req, uint64_t* ticket) {
  if (!srv || !req || !ticket) return fail(ENVAR_EINVAL, "NULL argument");
  Server& S = srv->impl;
  envar_problem pb = req->problem;
  pb.precision = S.cfg.precision;
  pb.flags |= S.cfg.flags & ENVAR_FLAG_NO_GRAPHS;
  auto* r = new Request;
  int rc = make_plan(&pb, r->P);
  if (rc) {
    delete r;
    return rc;
  }
  if (!req->state_dev || !req->controls || req->n_rows < 1 || req->horizon < 1 || req->m != r->P.m) {
    delete r;
    return fail(ENVAR_EINVAL, "bad request (NULL pointer, n_rows/horizon < 1 or m mismatch)");
  }
  r->n = req->n_rows;
  r->horizon = req->horizon;
  r->L = req_layout(r->P, r->n);
  if (r->L.total > S.alloc.size) {
    delete r;
    return fail(ENVAR_ENOMEM, "request needs %zu bytes, the pool holds %zu", r->L.total, S.alloc.size);
  }
  r->controls.assign(req->controls, req->controls + (size_t)r->n * r->P.m);
  r->job.P = r->P;
  r->job.w = make_ws(r->P, r->n);
  r->job.state = req->state_dev;
  r->job.nmem = r->n;
  r->job.horizon = r->horizon;
  r->st.cell_steps = (double)r->P.ncells * r->horizon * r->n;
  if (hipHostMalloc((void**)&r->J_pinned, (size_t)r->n * (2 + STATS_STRIDE) * 8, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming) != hipSuccess) {
    if (r->J_pinned) (void)hipHostFree(r->J_pinned);
    delete r;
    return fail(ENVAR_EDEVICE, "cannot allocate the request's host staging");
  }
  std::lock_guard<std::mutex> lk(S.mu);
  if (S.stop) {
    (void)hipHostFree(r->J_pinned);
    (void)hipEventDestroy(r->done_ev);
    delete r;
    return fail(ENVAR_ECANCELLED, "server stopped: %s", S.err.c_str());
  }
  if ((int)S.queue.size() >= S.cfg.max_queue) {
    (void)hipHostFree(r->J_pinned);
    (void)hipEventDestroy(r->done_ev);
    delete r;
    return fail(ENVAR_EBUSY, "queue full (%d requests)", S.cfg.max_queue);
  }
  r->ticket = S.next_ticket++;
  r->st.submit_s = S.now();
  S.table[r->ticket] = r;
  S.queue.push_back(r);
  *ticket = r->ticket;
  S.cv_work.notify_one();
  return ENVAR_OK;
}

int envar_wait(envar_server* srv, uint64_t ticket, double timeout_s, double* J_host, envar_request_stats* stats) {
  if (!srv) return fail(ENVAR_EINVAL, "NULL server");
  Server& S = srv->impl;
  std::unique_lock<std::mutex> lk(S.mu);
  auto it = S.table.find(ticket);
  if (it == S.table.end()) return fail(ENVAR_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second;
  auto ready = [&] { return r->phase == 3 || S.stop; };
  if (timeout_s < 0)
    S.cv_done.wait(lk, ready);
  else if (!S.cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready))
    return fail(ENVAR_ETIMEOUT, "ticket %llu not done after %.3f s", (unsigned long long)ticket, timeout_s);
  if (r->phase != 3) return fail(ENVAR_ECANCELLED, "server stopped: %s", S.err.c_str());
  if (J_host) std::copy(r->J.begin(), r->J.end(), J_host);
  if (stats) *stats = r->st;
  const int status = r->st.status;
  const int unconv = r->st.unconverged;
  S.table.erase(it);
  (void)hipHostFree(r->J_pinned);
  (void)hipEventDestroy(r->done_ev);
  delete r;
  const unsigned long long t = (unsigned long long)ticket;
  switch (status) {
    case ENVAR_OK:
      return ENVAR_OK;
    case ENVAR_EDIVERGED:
      return fail(ENVAR_EDIVERGED, "a cost of ticket %llu is non-finite", t);
    case ENVAR_EUNCONVERGED:
      return fail(ENVAR_EUNCONVERGED, "ticket %llu: %d member-step(s) stopped at the pass cap before div_tol", t,
                  unconv);
    default:
      return fail(status, "ticket %llu failed on the device: %s", t, S.err.c_str());
  }
}

int envar_server_destroy(envar_server* srv) {
  if (!srv) return ENVAR_OK;
  Server& S = srv->impl;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stop = true;
    S.cv_work.notify_all();
    S.cv_done.notify_all();
  }
  if (S.worker.joinable()) S.worker.join();
  for (auto& kv : S.table) {
    Request* r = kv.second;
    if (r->J_pinned) (void)hipHostFree(r->J_pinned);
    if (r->done_ev) (void)hipEventDestroy(r->done_ev);
    delete r;
  }
  S.table.clear();
  (void)hipStreamDestroy(S.s);
  delete srv;
  return ENVAR_OK;
}

}  // extern "C"
