// Host side of the C ABI declared in include/ising.h: validation, packing of
// the layered systems into device tables, tiling, launch sequencing.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ising.h"
#include "internal.h"
#include "mlp.h"

using namespace ising;

static thread_local std::string g_err;

static int32_t fail(int32_t code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

static int32_t hip_fail(hipError_t e, const char *where) {
  return fail(ISING_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(expr, where)                     \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

extern "C" const char *ising_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// Host-only helpers
// ---------------------------------------------------------------------------
extern "C" int32_t ising_threshold_row(double beta, int32_t dmax, uint32_t *thr) {
  if (!thr || dmax < 0 || dmax > 1023) return fail(ISING_E_INVAL, "threshold_row: bad arguments");
  if (!(beta > 0.0) || !isfinite(beta)) return fail(ISING_E_RANGE, "threshold_row: beta must be > 0");
  thr[0] = 0xffffffffu;
  for (int32_t d = 1; d <= dmax; ++d) {
    // u * 2^-32 < p  <=>  u < ceil(2^32 p)  <=>  u <= ceil(2^32 p) - 1 for integer u.
    const double p = exp(-2.0 * beta * (double)d);
    const double t = ceil(ldexp(p, 32));  // exact: scaling by 2^32, ceil of a double
    const uint64_t ti = (uint64_t)t;      // 1 .. 2^32
    thr[d] = (uint32_t)(ti - 1u);
  }
  return ISING_OK;
}

// e^x as Section 2.4 / Figure 7 approximate it, in FP32: scale x by 2^23 log2 e
// (fast) or 2^25 log2 e (accurate), round to the nearest integer, add the bit
// pattern of 1.0f, read the result as a float and multiply by 2 ln^2 2; the
// accurate form then takes the 4th root (two IEEE square roots here).  Below
// the valid range (-126 ln 2, resp. -31.5 ln 2) the value is 0.
static float exp_fig7(float x, int32_t kind) {
  const bool fast = kind == ISING_ACCEPT_FAST;
  const float lo = (fast ? -126.0f : -31.5f) * 0.69314718055994531f;
  if (x < lo) return 0.0f;
  const float mul = (float)((fast ? 8388608.0 : 33554432.0) * 1.4426950408889634);
  const int32_t bits = (int32_t)lrintf(x * mul) + 0x3F800000;
  float f;
  memcpy(&f, &bits, sizeof f);
  f *= (float)(2.0 * 0.69314718055994531 * 0.69314718055994531);
  return fast ? f : sqrtf(sqrtf(f));
}

extern "C" int32_t ising_acceptance_row(double beta, int32_t dmax, int32_t kind, uint32_t *thr) {
  if (kind == ISING_ACCEPT_EXACT) return ising_threshold_row(beta, dmax, thr);
  if (kind != ISING_ACCEPT_FAST && kind != ISING_ACCEPT_ACCURATE) return fail(ISING_E_INVAL, "unknown acceptance kind");
  if (!thr || dmax < 0 || dmax > 1023) return fail(ISING_E_INVAL, "acceptance_row: bad arguments");
  if (!(beta > 0.0) || !isfinite(beta)) return fail(ISING_E_RANGE, "acceptance_row: beta must be > 0");
  thr[0] = 0xffffffffu;
  for (int32_t d = 1; d <= dmax; ++d) {
    const float p = exp_fig7((float)(-2.0 * beta * (double)d), kind);
    const double t = ceil(ldexp((double)p, 32)) - 1.0;  // u <= t  <=>  u * 2^-32 < p (p > 0)
    thr[d] = t < 0.0 ? 0u : (t > 4294967295.0 ? 0xffffffffu : (uint32_t)t);
  }
  return ISING_OK;
}

// Threshold of a flip whose log weight change is -2x (two-field form): every
// flip with x <= 0 passes; otherwise u <= t  <=>  u * 2^-32 < p, p = exp(-2x)
// (or the Figure 7 approximation of it, on -2x rounded to FP32).
static uint32_t two_field_threshold(double x, int32_t kind) {
  if (x <= 0.0) return 0xffffffffu;
  if (kind == ISING_ACCEPT_EXACT) {
    const double t = ceil(ldexp(exp(-2.0 * x), 32));  // 1 .. 2^32 for 0 < 2x <= 700
    return (uint32_t)((uint64_t)t - 1u);
  }
  const float p = exp_fig7((float)(-2.0 * x), kind);
  const double t = ceil(ldexp((double)p, 32)) - 1.0;
  return t < 0.0 ? 0u : (t > 4294967295.0 ? 0xffffffffu : (uint32_t)t);
}

// x = a d_sp + c d_t, the two products rounded separately (no fused multiply-add),
// the order the swap rule and the sweep's specification use.
static double two_field_arg(double a, double c, int32_t dsp, int32_t dt) {
#pragma clang fp contract(off)
  const double xs = a * (double)dsp;
  const double xt = c * (double)dt;
  return xs + xt;
}

extern "C" int32_t ising_two_field_row(double a, double c, int32_t ds, int32_t dt, int32_t kind, uint32_t *thr) {
  if (!thr || ds < 0 || dt < 0 || (int64_t)(2 * ds + 1) * (2 * dt + 1) > kMaxTwoFieldRow)
    return fail(ISING_E_INVAL, "two_field_row: bad arguments");
  if (kind != ISING_ACCEPT_EXACT && kind != ISING_ACCEPT_FAST && kind != ISING_ACCEPT_ACCURATE)
    return fail(ISING_E_INVAL, "unknown acceptance kind");
  if (!isfinite(a) || !isfinite(c)) return fail(ISING_E_RANGE, "two_field_row: weights must be finite");
  if (2.0 * (fabs(a) * ds + fabs(c) * dt) > 700.0)
    return fail(ISING_E_RANGE, "two_field_row: 2(|a| ds + |c| dt) exceeds 700");
  const int32_t wt = 2 * dt + 1;
  for (int32_t i = -ds; i <= ds; ++i)
    for (int32_t j = -dt; j <= dt; ++j) thr[(i + ds) * wt + j + dt] = two_field_threshold(two_field_arg(a, c, i, j), kind);
  return ISING_OK;
}

extern "C" int32_t ising_trotter_weights(const double *beta, int32_t n, int32_t M, double gamma, double *a,
                                         double *c) {
  if (!beta || !a || !c || n < 0 || M < 1) return fail(ISING_E_INVAL, "trotter_weights: bad arguments");
  if (!(gamma > 0.0) || !isfinite(gamma)) return fail(ISING_E_RANGE, "trotter_weights: gamma must be > 0");
  for (int32_t k = 0; k < n; ++k) {
    if (!(beta[k] > 0.0) || !isfinite(beta[k])) return fail(ISING_E_RANGE, "trotter_weights: beta must be > 0");
    a[k] = beta[k] / (double)M;
    c[k] = -0.5 * log(tanh(beta[k] * gamma / (double)M));
  }
  return ISING_OK;
}

struct SysHost {
  int32_t S, M, ring, F, deg, dmax, K, cell, FW;
  int32_t ds = 0, dt = 0;  // two-field bounds: max |h| + sum |J in-slice|, max sum |J_tau| of a spin
  int32_t grid_L = 0, n_phases = 0;
  std::vector<uint16_t> cells;  // cell indices, phase by phase
  int32_t pc[5] = {0, 0, 0, 0, 0};
  std::vector<TmplSpin> tmpl;
  std::vector<uint32_t> fifo;  // (queue base << 8) | log2(depth) per template spin
  std::vector<uint16_t> lanes;  // sweep lane position -> template spin, by level offset
  std::vector<uint32_t> cellrec;  // grid templates: kCellRecWords words per template cell
  std::vector<double> beta;
};

static int32_t build_system(const ising_system_desc &d, int32_t idx, SysHost &out) {
  const int32_t S = d.spins_per_slice, M = d.n_slices;
  if (S < 1 || S > ISING_MAX_S) return fail(ISING_E_RANGE, "system %d: S=%d outside 1..%d", idx, S, ISING_MAX_S);
  if (M < 1) return fail(ISING_E_INVAL, "system %d: n_slices must be >= 1", idx);
  if ((int64_t)S * M > (1 << 22)) return fail(ISING_E_RANGE, "system %d: too many spins", idx);
  if (d.ring != 0 && d.ring != 1) return fail(ISING_E_INVAL, "system %d: ring must be 0 or 1", idx);
  if (d.ring && M < 3) return fail(ISING_E_RANGE, "system %d: a ring needs M >= 3", idx);
  if (d.n_edges < 0 || (d.n_edges > 0 && (!d.edge_u || !d.edge_v || !d.edge_J)))
    return fail(ISING_E_INVAL, "system %d: edge arrays", idx);
  if (!d.h) return fail(ISING_E_INVAL, "system %d: h is NULL", idx);
  if (M > 1 && !d.J_tau) return fail(ISING_E_INVAL, "system %d: J_tau is NULL with M > 1", idx);
  if (d.n_temps < 1 || d.n_temps > ISING_MAX_K)
    return fail(ISING_E_RANGE, "system %d: K=%d outside 1..%d", idx, d.n_temps, ISING_MAX_K);
  if (!d.beta) return fail(ISING_E_INVAL, "system %d: beta is NULL", idx);
  for (int32_t k = 0; k < d.n_temps; ++k)
    if (!(d.beta[k] > 0.0) || !isfinite(d.beta[k])) return fail(ISING_E_RANGE, "system %d: beta[%d] must be > 0", idx, k);

  std::vector<std::vector<std::pair<int32_t, int8_t>>> nb(S);
  std::set<std::pair<int32_t, int32_t>> seen;
  for (int32_t e = 0; e < d.n_edges; ++e) {
    int32_t a = d.edge_u[e], b = d.edge_v[e];
    if (a < 0 || a >= S || b < 0 || b >= S || a == b)
      return fail(ISING_E_INVAL, "system %d: edge %d (%d,%d) invalid", idx, e, a, b);
    if (!seen.insert({std::min(a, b), std::max(a, b)}).second)
      return fail(ISING_E_INVAL, "system %d: duplicate edge (%d,%d)", idx, a, b);
    nb[a].push_back({b, d.edge_J[e]});
    nb[b].push_back({a, d.edge_J[e]});
  }
  const int32_t ntau = M == 1 ? 0 : 2;  // worst case per spin (middle slices / ring)
  out.S = S;
  out.M = M;
  out.ring = d.ring;
  out.K = d.n_temps;
  out.deg = 0;
  out.dmax = 0;
  out.tmpl.assign(S, TmplSpin{});
  std::vector<int32_t> f(S, 0);
  int32_t F = 1;
  for (int32_t q = 0; q < S; ++q) {
    if ((int32_t)nb[q].size() > ISING_MAX_DEG || (int32_t)nb[q].size() + ntau > 8)
      return fail(ISING_E_RANGE, "system %d: spin %d has %d in-slice + %d tau neighbours (max 8)", idx, q,
                  (int)nb[q].size(), ntau);
    std::sort(nb[q].begin(), nb[q].end());
    int32_t fq = 0, bound = std::abs((int32_t)d.h[q]);
    for (auto &p : nb[q]) {
      if (p.first < q) fq = std::max(fq, f[p.first] + 1);
      bound += std::abs((int32_t)p.second);
    }
    const int32_t jt = M > 1 ? d.J_tau[q] : 0;
    out.ds = std::max(out.ds, bound);
    out.dt = std::max(out.dt, ntau * std::abs(jt));
    bound += ntau * std::abs(jt);
    if (bound > ISING_MAX_D)
      return fail(ISING_E_RANGE, "system %d: |h|+sum|J| = %d at spin %d exceeds %d", idx, bound, q, ISING_MAX_D);
    f[q] = fq;
    F = std::max(F, fq + 1);
    out.dmax = std::max(out.dmax, bound);
    out.deg = std::max(out.deg, (int32_t)nb[q].size());
    TmplSpin &t = out.tmpl[q];
    for (int j = 0; j < kMaxDeg; ++j) {
      t.nbr[j] = (int16_t)q;
      t.J[j] = 0;
    }
    for (size_t j = 0; j < nb[q].size(); ++j) {
      t.nbr[j] = (int16_t)nb[q][j].first;
      t.J[j] = nb[q][j].second;
    }
    t.h = d.h[q];
    t.Jtau = (int8_t)jt;
    t.f = (uint8_t)fq;
    t.deg = (uint8_t)nb[q].size();
    t.jpack = 0;
  }
  // Cell templates: every spin is joined to the four spins of the other half of
  // its aligned group of eight (a K4,4 unit cell); those four go first, in
  // partner order, with their 2J packed into one word.
  bool cell = S % 8 == 0;
  for (int32_t q = 0; q < S && cell; ++q) {
    const int32_t p0 = (q & ~7) + ((q & 4) ^ 4);
    for (int32_t i = 0; i < 4 && cell; ++i) {
      bool found = false;
      for (auto &p : nb[q]) found |= p.first == p0 + i;
      cell = found;
    }
  }
  out.cell = cell ? 1 : 0;
  if (cell) {
    for (int32_t q = 0; q < S; ++q) {
      const int32_t p0 = (q & ~7) + ((q & 4) ^ 4);
      std::vector<std::pair<int32_t, int8_t>> order;
      for (int32_t i = 0; i < 4; ++i)
        for (auto &p : nb[q])
          if (p.first == p0 + i) order.push_back(p);
      for (auto &p : nb[q])
        if (p.first < p0 || p.first >= p0 + 4) order.push_back(p);
      TmplSpin &t = out.tmpl[q];
      uint32_t pack = 0;
      for (size_t j = 0; j < order.size(); ++j) {
        t.nbr[j] = (int16_t)order[j].first;
        t.J[j] = order[j].second;
        if (j < 4) pack |= (uint32_t)(uint8_t)(int8_t)(2 * order[j].second) << (8 * j);
      }
      t.jpack = (int32_t)pack;
    }
  }
  if (F > 255) return fail(ISING_E_RANGE, "system %d: schedule depth %d exceeds 255", idx, F);
  out.F = F;
  // Sweep lanes: the columns in order of their level offset (ties in index
  // order).  A column is busy for M consecutive levels from f(q), so a
  // wavefront whose columns share nearly one offset idles on few levels; in
  // index order a wavefront of a Chimera template spans offsets y .. y + L.
  out.lanes.resize(S);
  for (int32_t q = 0; q < S; ++q) out.lanes[q] = (uint16_t)q;
  std::stable_sort(out.lanes.begin(), out.lanes.end(), [&](uint16_t a, uint16_t b) { return f[a] < f[b]; });
  // Uniform queues.  Slot k of column q's queue is word base(q) + 64 k: a
  // queue lives in one LDS bank.  The columns of 64 consecutive lane positions
  // (one wavefront) take 64 different banks, bank (l + r_w) mod 64 for
  // position l of the group, with a rotation r_w per group chosen so that the
  // banks' stacks stay even; a wavefront's queue reads then never conflict.
  out.fifo.assign(S, 0);
  {
    int32_t height[64] = {0};
    for (int32_t g0 = 0; g0 < S; g0 += 64) {
      int32_t best_r = 0, best_h = INT32_MAX;
      for (int32_t r = 0; r < 64; ++r) {
        int32_t hmax = 0;
        for (int32_t l = 0; l < 64 && g0 + l < S; ++l)
          hmax = std::max(hmax, height[(l + r) & 63] + fifo_depth(f[out.lanes[g0 + l]]));
        if (hmax < best_h) best_h = hmax, best_r = r;
      }
      for (int32_t l = 0; l < 64 && g0 + l < S; ++l) {
        const int32_t q = out.lanes[g0 + l], b = (l + best_r) & 63, dq = fifo_depth(f[q]);
        int32_t lg = 0;
        while ((1 << lg) < dq) ++lg;
        out.fifo[q] = ((uint32_t)(height[b] * 64 + b) << 8) | (uint32_t)lg;
        height[b] += dq;
      }
    }
    int32_t hmax = 0;
    for (int32_t b = 0; b < 64; ++b) hmax = std::max(hmax, height[b]);
    out.FW = hmax * 64;
  }
  // Grid of 8-spin cells (cell moves): S = 8 L^2, cell templates, and every
  // in-slice edge between two cells joins grid neighbours; then cells coloured
  // (y + x + m) mod 2 share no edge (on a ring of odd length the last slice
  // takes colours 2 and 3).
  out.grid_L = 0;
  if (cell) {
    int32_t L = 1;
    while (8 * L * L < S) ++L;
    bool grid = 8 * L * L == S && (int64_t)L * L * M <= 65535;
    for (int32_t e = 0; e < d.n_edges && grid; ++e) {
      const int32_t ca = d.edge_u[e] / 8, cb = d.edge_v[e] / 8;
      if (ca == cb) continue;
      const int32_t dy = std::abs(ca / L - cb / L), dx = std::abs(ca % L - cb % L);
      grid = dy + dx == 1;
    }
    if (grid) {
      out.grid_L = L;
      out.n_phases = (d.ring && M % 2 == 1) ? 4 : 2;
      std::vector<std::vector<uint16_t>> ph(out.n_phases);
      for (int32_t m = 0; m < M; ++m)
        for (int32_t y = 0; y < L; ++y)
          for (int32_t x = 0; x < L; ++x) {
            const int32_t col = (d.ring && M % 2 == 1 && m == M - 1) ? 2 + (y + x) % 2 : (y + x + m) % 2;
            ph[col].push_back((uint16_t)((m * L + y) * L + x));
          }
      out.cells.clear();
      for (int32_t p = 0; p < out.n_phases; ++p) {
        out.pc[p] = (int32_t)out.cells.size();
        out.cells.insert(out.cells.end(), ph[p].begin(), ph[p].end());
      }
      for (int32_t p = out.n_phases; p < 5; ++p) out.pc[p] = (int32_t)out.cells.size();
      // cell records: the neighbours outside the cell, by direction and bit
      out.cellrec.assign((size_t)L * L * kCellRecWords, 0u);
      for (int32_t c = 0; c < L * L; ++c) {
        uint32_t *rec = out.cellrec.data() + (size_t)c * kCellRecWords;
        for (int32_t k = 0; k < 8; ++k) {
          const TmplSpin &t = out.tmpl[c * 8 + k];
          int32_t e = 0;
          for (int32_t j = 4; j < t.deg; ++j) {
            const int32_t nb = t.nbr[j], cn = nb >> 3;
            const int32_t dir = cn == c - L ? 0 : cn == c + L ? 1 : cn == c - 1 ? 2 : 3;
            const uint32_t ent = (uint32_t)(uint8_t)t.J[j] | ((uint32_t)(8 * dir + (nb & 7)) << 8);
            rec[2 * k + (e >> 1)] |= ent << (16 * (e & 1));
            ++e;
          }
          rec[16 + (k >> 2)] |= (uint32_t)(uint8_t)t.h << (8 * (k & 3));
          rec[18 + (k >> 2)] |= (uint32_t)(uint8_t)t.Jtau << (8 * (k & 3));
          if (k < 4) rec[20 + k] = (uint32_t)t.jpack;
        }
      }
    }
  }
  out.beta.assign(d.beta, d.beta + d.n_temps);
  return ISING_OK;
}

extern "C" int32_t ising_level_offsets(const ising_system_desc *sys, int32_t *f, int32_t *depth) {
  if (!sys || !f || !depth) return fail(ISING_E_INVAL, "level_offsets: NULL argument");
  SysHost h;
  int32_t rc = build_system(*sys, 0, h);
  if (rc) return rc;
  for (int32_t q = 0; q < h.S; ++q) f[q] = h.tmpl[q].f;
  *depth = h.F;
  return ISING_OK;
}

// ---------------------------------------------------------------------------
// Graph handle
// ---------------------------------------------------------------------------
struct ising_graph {
  int32_t n_sys = 0;
  int64_t R = 0, slots = 0, spin_words = 0, attempts = 0, max_levels = 0;
  int64_t cell_rows = 0, total_cells = 0;
  int32_t max_phases = 0;
  std::vector<SysInfo> sys;
  std::vector<Tile> tiles;
  std::vector<Bucket> buckets;
  std::vector<std::vector<int32_t>> bucket_sys;  // systems of each bucket
  std::vector<int32_t> walker_sys;
  std::vector<double> slot_beta;  // beta of every slot, in slot order
  bool ladder_all() const {
    if (two_field) return false;
    for (const Bucket &b : buckets)
      if (!b.ladder) return false;
    return !buckets.empty();
  }
  int32_t accept_kind = ISING_ACCEPT_EXACT;
  // two-field form: graph-wide bounds of d_sp and d_t, row words (0: rows too long)
  int32_t qds = 0, qdt = 0, qrow = 0;
  bool two_field = false;
  // layer-pair order: generator lanes, launch size, classes present ("" if supported)
  int64_t pair_lanes = 0;
  int32_t pair_threads = 0;
  size_t pair_lds = 0;
  uint32_t pair_classes = 0;
  std::string pair_why;
  std::vector<double> qa, qc;  // per slot, while the two-field form is on
  // LDS words of a walker slot for system s in the current form
  int32_t walker_words(int32_t s) const {
    const SysInfo &si = sys[s];
    return two_field ? walker_lds_words(si.S, si.WW, si.fifo_words, si.RS, std::max(qrow, kThrRow), 5)
                     : walker_lds_words(si.S, si.WW, si.fifo_words, si.RS);
  }
  DevTables dev{};
  size_t bytes = 0;
  // With several buckets, bucket b > 0 is launched on side[b - 1] (forked from
  // and joined back to the caller's stream), so the buckets of one sweep run
  // side by side and each one's tail overlaps the others.
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;  // ev[0]: fork; ev[b]: bucket b done
  ~ising_graph() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipStream_t q : side) (void)hipStreamDestroy(q);
  }
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t sys, tmpl, fifo, lanes, thr, beta, tiles, wsys, cells, rtiles, cellrec, qthr, qa, qc, total;
};

// Device tables.  Room for one tile per walker, so any launch shape can be
// installed later without reallocating.
static Layout layout_for(int64_t n_sys, int64_t n_tmpl, int64_t slots, int64_t n_tiles, int64_t R, int64_t n_cells,
                         int64_t cell_rows, int64_t n_cellrec, int64_t qrow) {
  Layout L{};
  size_t o = 0;
  n_tiles = std::max(n_tiles, R);
  L.sys = o;
  o = align256(o + sizeof(SysInfo) * n_sys);
  L.tmpl = o;
  o = align256(o + sizeof(TmplSpin) * n_tmpl);
  L.fifo = o;
  o = align256(o + sizeof(uint32_t) * n_tmpl);
  L.lanes = o;
  o = align256(o + sizeof(uint16_t) * n_tmpl);
  L.thr = o;
  o = align256(o + sizeof(uint32_t) * kThrRow * slots);
  L.beta = o;
  o = align256(o + sizeof(double) * slots);
  L.tiles = o;
  o = align256(o + sizeof(Tile) * n_tiles);
  L.wsys = o;
  o = align256(o + sizeof(int32_t) * R);
  L.cells = o;
  o = align256(o + sizeof(uint16_t) * std::max<int64_t>(n_cells, 1));
  L.rtiles = o;
  o = align256(o + sizeof(int32_t) * std::max<int64_t>(cell_rows / 64, 1));
  L.cellrec = o;
  o = align256(o + sizeof(uint32_t) * std::max<int64_t>(n_cellrec, 1));
  L.qthr = o;  // two-field threshold rows
  o = align256(o + sizeof(uint32_t) * std::max<int64_t>(qrow * slots, 1));
  L.qa = o;
  o = align256(o + sizeof(double) * slots);
  L.qc = o;
  o = align256(o + sizeof(double) * slots);
  L.total = o;
  return L;
}

// Launch shape of a bucket: `tpw` threads per walker (a power of two; each
// thread owns ceil(S/tpw) <= 8 columns) and G walkers per workgroup.
static int32_t shape_bucket(Bucket &b, int32_t tpw, int32_t G, int32_t Kmax, bool allow_ladder = true) {
  if (tpw < 1 || (tpw & (tpw - 1)) != 0 || tpw > 1024) return fail(ISING_E_RANGE, "tpw must be a power of two <= 1024");
  const int32_t need = (b.S + tpw - 1) / tpw;
  int32_t cpt = 1;
  while (cpt < need) cpt <<= 1;
  if (cpt > 8) return fail(ISING_E_RANGE, "tpw=%d leaves %d columns per thread (max 8)", tpw, need);
  if (G < 1) return fail(ISING_E_RANGE, "G must be >= 1");
  G = std::min(G, Kmax);
  if ((int64_t)G * tpw > 1024) return fail(ISING_E_RANGE, "G*tpw exceeds 1024 threads");
  size_t lds = (size_t)G * b.walker_words * 4;
  if (lds > 160 * 1024) return fail(ISING_E_RANGE, "launch shape needs %zu bytes of LDS (> 160 KiB)", lds);
  // A workgroup that holds whole systems (G >= Kmax) runs their swap rounds
  // itself when the swap state fits next to the walkers.
  const bool ladder = allow_ladder && G >= Kmax && Kmax <= 256 && tpw <= 64 &&
                      lds + (size_t)kLadderWords * 4 <= 160 * 1024;
  if (ladder) lds += (size_t)kLadderWords * 4;
  b.tpw = tpw;
  b.cpt = cpt;
  b.G = G;
  b.kmax = Kmax;
  b.ladder = ladder ? 1 : 0;
  b.threads = std::max(64, ((G * tpw + 63) / 64) * 64);
  b.lds = lds;
  return ISING_OK;
}

// Default shape (measured on MI355X for 8x8 and 4x4 cell templates): at most
// two columns per thread, up to 256 threads and ~40 KiB of LDS per workgroup.
// Small systems whose whole ladder fits one workgroup take G = Kmax, so their
// sweeps and swap rounds run in one launch.
static void default_shape(int32_t S, int32_t walker_words, int32_t Kmax, int32_t &tpw, int32_t &G,
                          bool allow_ladder = true) {
  int32_t p = 8;
  while (p < S) p <<= 1;
  tpw = p >= 256 ? p / 2 : p;
  G = std::max(1, 256 / tpw);
  while (G > 1 && (size_t)G * walker_words * 4 > 40 * 1024) --G;
  if (allow_ladder && G < Kmax && tpw <= 64 && (int64_t)Kmax * tpw <= 1024 &&
      ((size_t)Kmax * walker_words + kLadderWords) * 4 <= 160 * 1024)
    G = Kmax;
}

static void tile_bucket(ising_graph &g, Bucket &b, const std::vector<int32_t> &systems) {
  b.tile0 = (int32_t)g.tiles.size();
  for (int32_t s : systems)
    for (int32_t w0 = 0; w0 < g.sys[s].K; w0 += b.G)
      g.tiles.push_back(Tile{s, w0, std::min(b.G, g.sys[s].K - w0), 0});
  b.ntiles = (int32_t)g.tiles.size() - b.tile0;
}

static int32_t plan(const std::vector<SysHost> &hs, ising_graph &g) {
  g.n_sys = (int32_t)hs.size();
  g.sys.resize(hs.size());
  int64_t walker = 0, slot = 0, word = 0, tmpl = 0, cl = 0, cb = 0;
  for (size_t s = 0; s < hs.size(); ++s) {
    const SysHost &h = hs[s];
    SysInfo &si = g.sys[s];
    si.S = h.S;
    si.M = h.M;
    si.ring = h.ring;
    si.F = h.F;
    const int32_t sw = (h.S + 31) / 32;
    si.RS = (sw > 1 && sw % 2 == 0) ? sw + 1 : sw;
    si.WW = si.RS * h.M;
    si.K = h.K;
    si.walker0 = (int32_t)walker;
    si.spin_word0 = word;
    si.tmpl0 = (int32_t)tmpl;
    si.thr0 = (int32_t)slot;
    si.slot0 = (int32_t)slot;
    si.deg = h.deg;
    si.cell = h.cell;
    si.nx = h.deg - (h.cell ? 4 : 0);
    si.fifo_words = h.FW;
    si.cb0 = (int32_t)cb;
    si.grid_L = h.grid_L;
    si.n_phases = h.n_phases;
    si.cl0 = (int32_t)cl;
    for (int p = 0; p < 5; ++p) si.pc[p] = h.pc[p];
    si.rows = 0;
    for (int p = 0; p < h.n_phases; ++p) si.rows = std::max(si.rows, h.pc[p + 1] - h.pc[p]);
    // layer-pair order: one generator lane per pair of slices of every walker
    si.pl0 = (int32_t)std::min<int64_t>(g.pair_lanes, INT32_MAX);
    {
      const int64_t lanes = (int64_t)h.K * (h.M / 2);
      const size_t lds = ((size_t)h.K * pair_walker_words(si.WW) + kLadderWords + 3 * (size_t)h.S) * 4;
      if (g.pair_why.empty()) {
        if (h.M < 2 || h.M % 2)
          g.pair_why = "system " + std::to_string(s) + " has an odd number of slices";
        else if (!h.cell || h.deg > 6)
          g.pair_why = "system " + std::to_string(s) + " is not a grid of K4,4 cells";
        else if (lanes > 1024)
          g.pair_why = "system " + std::to_string(s) + " needs more than 1024 lanes (K * M/2)";
        else if (lds > 160 * 1024)
          g.pair_why = "system " + std::to_string(s) + " needs more than 160 KiB of LDS";
      }
      g.pair_lanes += lanes;
      g.pair_threads = std::max<int32_t>(g.pair_threads, (int32_t)((lanes + 63) / 64 * 64));
      g.pair_lds = std::max(g.pair_lds, lds);
      g.pair_classes |= 1u << h.ring;
    }
    si.row0 = g.cell_rows;  // a multiple of 64: a 64-row tile of cell moves lies in one system
    si.cell0 = g.total_cells;
    g.cell_rows += ((int64_t)si.rows * h.K + 63) / 64 * 64;
    g.total_cells += h.grid_L ? (int64_t)h.grid_L * h.grid_L * h.M * h.K : 0;
    g.max_phases = std::max(g.max_phases, h.n_phases);
    cl += (int64_t)h.cells.size();
    cb += (int64_t)h.cellrec.size() / kCellRecWords;
    walker += h.K;
    slot += h.K;
    word += (int64_t)si.WW * h.K;
    tmpl += h.S;
    g.attempts += (int64_t)h.S * h.M * h.K;
    g.max_levels = std::max<int64_t>(g.max_levels, h.M + h.F - 1);
    for (int32_t k = 0; k < h.K; ++k) g.walker_sys.push_back((int32_t)s);
  }
  if (walker > INT32_MAX || slot > INT32_MAX) return fail(ISING_E_RANGE, "too many walkers");
  if (g.pair_why.empty() && g.pair_lanes > INT32_MAX) g.pair_why = "too many generator lanes";
  for (const SysHost &h : hs) {
    g.qds = std::max(g.qds, h.ds);
    g.qdt = std::max(g.qdt, h.dt);
  }
  {
    const int64_t qr = (int64_t)(2 * g.qds + 1) * (2 * g.qdt + 1);
    g.qrow = qr <= kMaxTwoFieldRow ? (int32_t)qr : 0;
  }
  g.R = walker;
  g.slots = slot;
  g.spin_words = word;
  // Buckets: systems sharing (S, ring, cell, neighbour class); one launch each.
  std::map<std::tuple<int32_t, int32_t, int32_t, int32_t>, std::vector<int32_t>> groups;
  for (size_t s = 0; s < hs.size(); ++s) {
    const int32_t nx = g.sys[s].nx;
    const int32_t nc = nx <= 0 ? 0 : nx <= 2 ? 2 : nx <= 4 ? 4 : nx <= 6 ? 6 : 8;
    groups[{hs[s].S, hs[s].ring, hs[s].cell, nc}].push_back((int32_t)s);
  }
  for (auto &kv : groups) {
    Bucket b{};
    b.S = std::get<0>(kv.first);
    b.ring = std::get<1>(kv.first);
    b.cell = std::get<2>(kv.first);
    b.nx = std::get<3>(kv.first);
    int32_t maxw = 0, Kmax = 1;
    for (int32_t s : kv.second) {
      maxw = std::max(maxw, g.walker_words(s));
      Kmax = std::max(Kmax, g.sys[s].K);
    }
    b.walker_words = maxw;
    int32_t tpw, G;
    default_shape(b.S, maxw, Kmax, tpw, G);
    int32_t rc = shape_bucket(b, tpw, G, Kmax);
    if (rc) return rc;
    tile_bucket(g, b, kv.second);
    g.buckets.push_back(b);
    g.bucket_sys.push_back(kv.second);
  }
  return ISING_OK;
}

static int32_t build_all(const ising_system_desc *sys, int32_t n_sys, std::vector<SysHost> &hs) {
  if (!sys || n_sys < 1) return fail(ISING_E_INVAL, "need at least one system");
  hs.resize(n_sys);
  for (int32_t s = 0; s < n_sys; ++s) {
    int32_t rc = build_system(sys[s], s, hs[s]);
    if (rc) return rc;
  }
  return ISING_OK;
}

extern "C" int32_t ising_graph_bytes(const ising_system_desc *sys, int32_t n_sys, size_t *dev_bytes) {
  if (!dev_bytes) return fail(ISING_E_INVAL, "dev_bytes is NULL");
  std::vector<SysHost> hs;
  int32_t rc = build_all(sys, n_sys, hs);
  if (rc) return rc;
  ising_graph g;
  rc = plan(hs, g);
  if (rc) return rc;
  int64_t ntm = 0, ncl = 0, ncr = 0;
  for (auto &h : hs) {
    ntm += h.S;
    ncl += (int64_t)h.cells.size();
    ncr += (int64_t)h.cellrec.size();
  }
  *dev_bytes = layout_for(n_sys, ntm, g.slots, (int64_t)g.tiles.size(), g.R, ncl, g.cell_rows, ncr, g.qrow).total;
  return ISING_OK;
}

extern "C" int32_t ising_load_graph(const ising_system_desc *sys, int32_t n_sys, void *dev_tables,
                                    size_t bytes, void *stream, ising_graph **out) {
  if (!out || !dev_tables) return fail(ISING_E_INVAL, "load_graph: NULL argument");
  if (((uintptr_t)dev_tables & 255u) != 0) return fail(ISING_E_INVAL, "dev_tables must be 256-byte aligned");
  *out = nullptr;
  std::vector<SysHost> hs;
  int32_t rc = build_all(sys, n_sys, hs);
  if (rc) return rc;
  ising_graph *g = new ising_graph();
  rc = plan(hs, *g);
  if (rc) {
    delete g;
    return rc;
  }
  int64_t ntm = 0, ncl = 0, ncr = 0;
  for (auto &h : hs) {
    ntm += h.S;
    ncl += (int64_t)h.cells.size();
    ncr += (int64_t)h.cellrec.size();
  }
  Layout L = layout_for(n_sys, ntm, g->slots, (int64_t)g->tiles.size(), g->R, ncl, g->cell_rows, ncr, g->qrow);
  if (bytes < L.total) {
    delete g;
    return fail(ISING_E_SIZE, "dev_tables has %zu bytes, needs %zu", bytes, L.total);
  }
  std::vector<uint8_t> host(L.total, 0);
  memcpy(host.data() + L.sys, g->sys.data(), sizeof(SysInfo) * g->sys.size());
  {
    TmplSpin *t = (TmplSpin *)(host.data() + L.tmpl);
    for (auto &h : hs) {
      memcpy(t, h.tmpl.data(), sizeof(TmplSpin) * h.S);
      t += h.S;
    }
    uint32_t *thr = (uint32_t *)(host.data() + L.thr);
    double *bt = (double *)(host.data() + L.beta);
    for (auto &h : hs)
      for (int32_t k = 0; k < h.K; ++k) {
        uint32_t row[kThrRow - kThrZero];
        rc = ising_threshold_row(h.beta[k], kThrRow - kThrZero - 1, row);
        if (rc) {
          delete g;
          return rc;
        }
        for (int32_t i = 0; i < kThrRow; ++i) thr[i] = i <= kThrZero ? 0xffffffffu : row[i - kThrZero];
        thr += kThrRow;
        *bt++ = h.beta[k];
        g->slot_beta.push_back(h.beta[k]);
      }
  }
  {
    uint32_t *fo = (uint32_t *)(host.data() + L.fifo);
    uint16_t *lo = (uint16_t *)(host.data() + L.lanes);
    for (auto &h : hs) {
      memcpy(fo, h.fifo.data(), sizeof(uint32_t) * h.S);
      memcpy(lo, h.lanes.data(), sizeof(uint16_t) * h.S);
      fo += h.S;
      lo += h.S;
    }
  }
  {
    uint16_t *co = (uint16_t *)(host.data() + L.cells);
    for (auto &h : hs) {
      memcpy(co, h.cells.data(), sizeof(uint16_t) * h.cells.size());
      co += h.cells.size();
    }
  }
  {
    uint32_t *cr = (uint32_t *)(host.data() + L.cellrec);
    for (auto &h : hs) {
      memcpy(cr, h.cellrec.data(), sizeof(uint32_t) * h.cellrec.size());
      cr += h.cellrec.size();
    }
  }
  {  // system of each 64-row tile of cell moves: the last system whose rows start at or before it
    int32_t *ts = (int32_t *)(host.data() + L.rtiles);
    int32_t sidx = 0;
    for (int64_t t = 0; t < g->cell_rows / 64; ++t) {
      while (sidx + 1 < n_sys && g->sys[sidx + 1].row0 <= t * 64) ++sidx;
      ts[t] = sidx;
    }
  }
  memcpy(host.data() + L.tiles, g->tiles.data(), sizeof(Tile) * g->tiles.size());
  memcpy(host.data() + L.wsys, g->walker_sys.data(), sizeof(int32_t) * g->walker_sys.size());
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(dev_tables, host.data(), L.total, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "load_graph copy");
  }
  uint8_t *base = (uint8_t *)dev_tables;
  g->dev.sys = (const SysInfo *)(base + L.sys);
  g->dev.tmpl = (const TmplSpin *)(base + L.tmpl);
  g->dev.thr = (const uint32_t *)(base + L.thr);
  g->dev.beta = (const double *)(base + L.beta);
  g->dev.tiles = (const Tile *)(base + L.tiles);
  g->dev.walker_sys = (const int32_t *)(base + L.wsys);
  g->dev.fifo = (const uint32_t *)(base + L.fifo);
  g->dev.lanes = (const uint16_t *)(base + L.lanes);
  g->dev.cells = (const uint16_t *)(base + L.cells);
  g->dev.tile_sys = (const int32_t *)(base + L.rtiles);
  g->dev.cellrec = (const uint32_t *)(base + L.cellrec);
  g->dev.qthr = (const uint32_t *)(base + L.qthr);
  g->dev.qa = (const double *)(base + L.qa);
  g->dev.qc = (const double *)(base + L.qc);
  g->dev.two_field = 0;
  g->dev.qrow = g->qrow;
  g->dev.qwt = 2 * g->qdt + 1;
  g->dev.qoff = g->qds * (2 * g->qdt + 1) + g->qdt;
  g->bytes = L.total;
  if (g->buckets.size() > 1) {
    for (size_t b = 0; b < g->buckets.size(); ++b) {
      hipEvent_t ev;
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e != hipSuccess) break;
      g->ev.push_back(ev);
      if (b == 0) continue;
      hipStream_t q;
      e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);  // default priority
      if (e != hipSuccess) break;
      g->side.push_back(q);
    }
    if (e != hipSuccess) {
      delete g;
      return hip_fail(e, "load_graph: bucket streams");
    }
  }
  *out = g;
  return ISING_OK;
}

extern "C" void ising_free_graph(ising_graph *g) { delete g; }

// Two-field threshold rows of every slot for the current weights and flip-test
// variant (host -> device, then synchronise).
static int32_t upload_two_field_rows(ising_graph *g, hipStream_t st) {
  std::vector<uint32_t> rows((size_t)g->slots * g->qrow);
  for (int64_t k = 0; k < g->slots; ++k) {
    const int32_t rc = ising_two_field_row(g->qa[k], g->qc[k], g->qds, g->qdt, g->accept_kind,
                                           rows.data() + (size_t)k * g->qrow);
    if (rc) return rc;
  }
  HIP_TRY(hipMemcpyAsync((void *)g->dev.qthr, rows.data(), rows.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st),
          "two-field rows copy");
  HIP_TRY(hipStreamSynchronize(st), "two-field rows sync");
  return ISING_OK;
}

extern "C" int32_t ising_set_acceptance(ising_graph *g, int32_t kind, void *stream) {
  if (!g) return fail(ISING_E_INVAL, "set_acceptance: NULL graph");
  std::vector<uint32_t> rows((size_t)g->slots * kThrRow);
  for (size_t k = 0; k < g->slot_beta.size(); ++k) {
    uint32_t row[kThrRow - kThrZero];
    const int32_t rc = ising_acceptance_row(g->slot_beta[k], kThrRow - kThrZero - 1, kind, row);
    if (rc) return rc;
    for (int32_t i = 0; i < kThrRow; ++i) rows[k * kThrRow + i] = i <= kThrZero ? 0xffffffffu : row[i - kThrZero];
  }
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync((void *)g->dev.thr, rows.data(), rows.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st),
          "set_acceptance copy");
  HIP_TRY(hipStreamSynchronize(st), "set_acceptance sync");
  g->accept_kind = kind;
  if (g->two_field) return upload_two_field_rows(g, st);
  return ISING_OK;
}

// Launch shapes after a change of the walker slot size: default shape per
// bucket (tuned shapes are dropped), tiles rebuilt and uploaded.
static int32_t reshape_all(ising_graph *g, hipStream_t st) {
  for (size_t bi = 0; bi < g->buckets.size(); ++bi) {
    Bucket &b = g->buckets[bi];
    int32_t maxw = 0, Kmax = 1;
    for (int32_t s : g->bucket_sys[bi]) {
      maxw = std::max(maxw, g->walker_words(s));
      Kmax = std::max(Kmax, g->sys[s].K);
    }
    b.walker_words = maxw;
    int32_t tpw, G;
    default_shape(b.S, maxw, Kmax, tpw, G, !g->two_field);
    int32_t rc = shape_bucket(b, tpw, G, Kmax, !g->two_field);
    if (rc) return rc;
  }
  g->tiles.clear();
  for (size_t i = 0; i < g->buckets.size(); ++i) tile_bucket(*g, g->buckets[i], g->bucket_sys[i]);
  HIP_TRY(hipMemcpyAsync((void *)g->dev.tiles, g->tiles.data(), sizeof(Tile) * g->tiles.size(),
                         hipMemcpyHostToDevice, st),
          "reshape tiles");
  HIP_TRY(hipStreamSynchronize(st), "reshape sync");
  return ISING_OK;
}

extern "C" int32_t ising_set_two_field(ising_graph *g, const double *a, const double *c, void *stream) {
  if (!g) return fail(ISING_E_INVAL, "set_two_field: NULL graph");
  hipStream_t st = (hipStream_t)stream;
  if (!a && !c) {  // back to the one-field form
    if (!g->two_field) return ISING_OK;
    g->two_field = false;
    g->dev.two_field = 0;
    g->qa.clear();
    g->qc.clear();
    return reshape_all(g, st);
  }
  if (!a || !c) return fail(ISING_E_INVAL, "set_two_field: give both weight arrays or neither");
  if (g->qrow == 0)
    return fail(ISING_E_RANGE, "set_two_field: threshold rows of (2*%d+1)*(2*%d+1) words exceed %d", g->qds, g->qdt,
                kMaxTwoFieldRow);
  for (const Bucket &b : g->buckets)
    if (!b.cell) return fail(ISING_E_RANGE, "set_two_field: every template must be a grid of K4,4 cells");
  for (int64_t k = 0; k < g->slots; ++k) {
    if (!isfinite(a[k]) || !isfinite(c[k])) return fail(ISING_E_RANGE, "set_two_field: weight %lld not finite", (long long)k);
    if (2.0 * (fabs(a[k]) * g->qds + fabs(c[k]) * g->qdt) > 700.0)
      return fail(ISING_E_RANGE, "set_two_field: slot %lld: 2(|a| d_sp + |c| d_t) may exceed 700", (long long)k);
  }
  g->qa.assign(a, a + g->slots);
  g->qc.assign(c, c + g->slots);
  HIP_TRY(hipMemcpyAsync((void *)g->dev.qa, a, sizeof(double) * g->slots, hipMemcpyHostToDevice, st), "two-field copy");
  HIP_TRY(hipMemcpyAsync((void *)g->dev.qc, c, sizeof(double) * g->slots, hipMemcpyHostToDevice, st), "two-field copy");
  int32_t rc = upload_two_field_rows(g, st);
  if (rc) return rc;
  const bool was = g->two_field;
  g->two_field = true;
  g->dev.two_field = 1;
  return was ? ISING_OK : reshape_all(g, st);
}

extern "C" int32_t ising_n_buckets(const ising_graph *g) { return g ? (int32_t)g->buckets.size() : 0; }

extern "C" int32_t ising_bucket_info(const ising_graph *g, int32_t bucket, int64_t *out, int32_t n) {
  if (!g || !out || bucket < 0 || bucket >= (int32_t)g->buckets.size())
    return fail(ISING_E_INVAL, "bucket_info: bad arguments");
  const Bucket &b = g->buckets[bucket];
  int64_t walkers = 0, attempts = 0;
  for (int32_t s : g->bucket_sys[bucket]) {
    walkers += g->sys[s].K;
    attempts += (int64_t)g->sys[s].K * g->sys[s].S * g->sys[s].M;
  }
  const int64_t v[11] = {b.S, (int64_t)g->bucket_sys[bucket].size(), walkers, attempts, b.tpw, b.G,
                         b.cpt, b.threads, (int64_t)b.lds, b.ntiles, b.ladder};
  for (int32_t i = 0; i < n && i < 11; ++i) out[i] = v[i];
  return ISING_OK;
}

extern "C" int32_t ising_set_launch(ising_graph *g, int32_t bucket, int32_t tpw, int32_t walkers_per_group,
                                    void *stream) {
  if (!g || bucket < 0 || bucket >= (int32_t)g->buckets.size())
    return fail(ISING_E_INVAL, "set_launch: bad bucket");
  Bucket b = g->buckets[bucket];
  int32_t Kmax = 1;
  for (int32_t s : g->bucket_sys[bucket]) Kmax = std::max(Kmax, g->sys[s].K);
  int32_t rc = shape_bucket(b, tpw, walkers_per_group, Kmax, !g->two_field);
  if (rc) return rc;
  g->buckets[bucket] = b;
  g->tiles.clear();
  for (size_t i = 0; i < g->buckets.size(); ++i) tile_bucket(*g, g->buckets[i], g->bucket_sys[i]);
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync((void *)g->dev.tiles, g->tiles.data(), sizeof(Tile) * g->tiles.size(),
                         hipMemcpyHostToDevice, st),
          "set_launch copy");
  HIP_TRY(hipStreamSynchronize(st), "set_launch sync");
  return ISING_OK;
}

extern "C" int32_t ising_graph_info(const ising_graph *g, int64_t *out, int32_t n) {
  if (!g || !out || n < 0) return fail(ISING_E_INVAL, "graph_info: bad arguments");
  const int64_t v[6] = {g->n_sys, g->R, g->slots, g->spin_words, g->attempts, g->max_levels};
  for (int32_t i = 0; i < n && i < 6; ++i) out[i] = v[i];
  return ISING_OK;
}

extern "C" int32_t ising_spin_layout(const ising_graph *g, int64_t *spin_word, int32_t *row_words) {
  if (!g || !spin_word || !row_words) return fail(ISING_E_INVAL, "spin_layout: NULL argument");
  for (int32_t s = 0; s < g->n_sys; ++s) {
    const SysInfo &si = g->sys[s];
    row_words[s] = si.RS;
    for (int32_t k = 0; k < si.K; ++k) spin_word[si.walker0 + k] = si.spin_word0 + (int64_t)k * si.WW;
  }
  return ISING_OK;
}

extern "C" int32_t ising_state_sizes(const ising_graph *g, int64_t *c) {
  if (!g || !c) return fail(ISING_E_INVAL, "state_sizes: NULL argument");
  c[0] = g->spin_words;
  c[1] = g->R * kMtN;
  c[2] = g->R;
  c[3] = g->R;
  c[4] = g->slots;
  c[5] = (int64_t)g->n_sys * kMtN;
  c[6] = g->R;
  c[7] = g->slots;
  c[8] = g->slots;
  c[9] = ISING_N_STATS;
  c[10] = 2 * g->R;
  c[11] = g->R;
  return ISING_OK;
}

static int32_t check_state(const ising_state *st) {
  if (!st || !st->spins || !st->mt || !st->energy || !st->temp_of || !st->walker_at || !st->swap_mt ||
      !st->flips || !st->swap_att || !st->swap_acc || !st->stats || !st->wsteps || !st->bond)
    return fail(ISING_E_INVAL, "state has a NULL buffer");
  return ISING_OK;
}

static DevState dev_state(const ising_state *st) {
  return DevState{st->spins, st->mt, st->energy, st->temp_of, st->walker_at, st->swap_mt,
                  st->flips, st->swap_att, st->swap_acc, st->stats, st->wsteps, st->bond};
}

extern "C" int32_t ising_init_state(const ising_graph *g, ising_state *st, const uint32_t *walker_seeds,
                                    const uint32_t *swap_seeds, void *stream) {
  if (!g || !walker_seeds || !swap_seeds) return fail(ISING_E_INVAL, "init_state: NULL argument");
  int32_t rc = check_state(st);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  DevState d = dev_state(st);
  // Seeds go to word 0 of each window; the seed kernel expands them.
  HIP_TRY(hipMemcpy2DAsync(st->mt, kMtN * sizeof(uint32_t), walker_seeds, sizeof(uint32_t), sizeof(uint32_t),
                           (size_t)g->R, hipMemcpyHostToDevice, s),
          "init_state seeds");
  HIP_TRY(hipMemcpy2DAsync(st->swap_mt, kMtN * sizeof(uint32_t), swap_seeds, sizeof(uint32_t),
                           sizeof(uint32_t), (size_t)g->n_sys, hipMemcpyHostToDevice, s),
          "init_state swap seeds");
  HIP_TRY(hipStreamSynchronize(s), "init_state sync");
  HIP_TRY(launch_seed(d, (int32_t)g->R, g->n_sys, s), "seed kernel");
  HIP_TRY(hipMemsetAsync(st->flips, 0, sizeof(uint64_t) * g->R, s), "init_state clear");
  HIP_TRY(hipMemsetAsync(st->swap_att, 0, sizeof(uint64_t) * g->slots, s), "init_state clear");
  HIP_TRY(hipMemsetAsync(st->swap_acc, 0, sizeof(uint64_t) * g->slots, s), "init_state clear");
  HIP_TRY(hipMemsetAsync(st->stats, 0, sizeof(uint64_t) * ISING_N_STATS, s), "init_state clear");
  HIP_TRY(hipMemsetAsync(st->wsteps, 0, sizeof(uint64_t) * 2 * g->R, s), "init_state clear");
  HIP_TRY(launch_labels(g->dev, d, (int32_t)g->R, g->n_sys, s), "labels kernel");
  for (const Bucket &b : g->buckets) HIP_TRY(launch_sweep(g->dev, d, b, 0, 1, s), "initial spins");
  HIP_TRY(launch_observables(g->dev, d, (int32_t)g->R, nullptr, 1, s), "initial energies");
  st->sweeps = 0;
  st->rounds = 0;
  return ISING_OK;
}

// Enqueue n_sweeps sweeps (and the swap rounds due) starting from the
// counters *sweeps / *rounds, advancing them.
// Launch every bucket (bucket b > 0 on side stream b - 1 when there are several,
// joined back to s).
static int32_t launch_buckets(const ising_graph *g, const DevState &d, int32_t n, LadderArgs la, hipStream_t s) {
  if (g->side.empty()) {
    for (const Bucket &b : g->buckets) HIP_TRY(launch_sweep(g->dev, d, b, n, 0, s, la), "sweep kernel");
    return ISING_OK;
  }
  HIP_TRY(hipEventRecord(g->ev[0], s), "fork");
  for (size_t b = 1; b < g->buckets.size(); ++b) {
    HIP_TRY(hipStreamWaitEvent(g->side[b - 1], g->ev[0], 0), "fork wait");
    HIP_TRY(launch_sweep(g->dev, d, g->buckets[b], n, 0, g->side[b - 1], la), "sweep kernel");
    HIP_TRY(hipEventRecord(g->ev[b], g->side[b - 1]), "join record");
  }
  HIP_TRY(launch_sweep(g->dev, d, g->buckets[0], n, 0, s, la), "sweep kernel");
  for (size_t b = 1; b < g->buckets.size(); ++b) HIP_TRY(hipStreamWaitEvent(s, g->ev[b], 0), "join");
  return ISING_OK;
}

static int32_t enqueue_sweeps(const ising_graph *g, const DevState &d, int64_t *sweeps, int64_t *rounds,
                              int32_t n_sweeps, int32_t swap_every, int32_t *e_series, hipStream_t s) {
  if (swap_every > 0 && !e_series && n_sweeps > 0 && g->ladder_all()) {
    // every system's ladder sits in one workgroup: sweeps and swap rounds in one launch
    const LadderArgs la{swap_every, 0, *sweeps, *rounds};
    int32_t rc = launch_buckets(g, d, n_sweeps, la, s);
    if (rc) return rc;
    *rounds += (*sweeps + n_sweeps) / swap_every - *sweeps / swap_every;
    *sweeps += n_sweeps;
    return ISING_OK;
  }
  int32_t done = 0;
  while (done < n_sweeps) {
    // Sweeps until the next swap round (or the end, or the next record).
    int32_t seg = n_sweeps - done;
    if (swap_every > 0) {
      const int64_t to_swap = swap_every - (*sweeps % swap_every);
      seg = (int32_t)std::min<int64_t>(seg, to_swap);
    }
    if (e_series) seg = 1;
    int32_t rc = launch_buckets(g, d, seg, LadderArgs{0, 0, 0, 0}, s);
    if (rc) return rc;
    *sweeps += seg;
    done += seg;
    int32_t *row = e_series ? e_series + (size_t)(done - 1) * g->slots : nullptr;
    if (swap_every > 0 && *sweeps % swap_every == 0) {
      HIP_TRY(launch_swap(g->dev, d, g->n_sys, (int32_t)(*rounds & 1), row, s), "swap kernel");
      *rounds += 1;
    } else if (row) {
      HIP_TRY(launch_record(g->dev, d, g->n_sys, row, s), "record kernel");
    }
  }
  return ISING_OK;
}

extern "C" int32_t ising_sweep(const ising_graph *g, ising_state *st, int32_t n_sweeps, int32_t swap_every,
                               int32_t *e_series, void *stream) {
  if (!g) return fail(ISING_E_INVAL, "sweep: NULL graph");
  int32_t rc = check_state(st);
  if (rc) return rc;
  if (n_sweeps < 0 || swap_every < 0) return fail(ISING_E_INVAL, "sweep: negative count");
  if (st->sweeps < 0) return fail(ISING_E_STATE, "sweep: state not initialised");
  return enqueue_sweeps(g, dev_state(st), &st->sweeps, &st->rounds, n_sweeps, swap_every, e_series,
                        (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Captured sweep loops (hipGraph)
// ---------------------------------------------------------------------------
struct ising_replay {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t sweeps0 = 0, rounds0 = 0, dsweeps = 0, drounds = 0;
  int32_t swap_every = 0;
  DevState dev{};
};

extern "C" int32_t ising_capture(const ising_graph *g, const ising_state *st, int32_t n_sweeps,
                                 int32_t swap_every, int32_t *e_series, void *stream, ising_replay **out) {
  if (!g || !out) return fail(ISING_E_INVAL, "capture: NULL argument");
  int32_t rc = check_state(st);
  if (rc) return rc;
  if (n_sweeps < 1 || swap_every < 0) return fail(ISING_E_INVAL, "capture: need n_sweeps >= 1");
  if (!stream) return fail(ISING_E_INVAL, "capture: needs a non-default stream");
  if (st->sweeps < 0) return fail(ISING_E_STATE, "capture: state not initialised");
  hipStream_t s = (hipStream_t)stream;
  ising_replay *r = new ising_replay();
  r->sweeps0 = st->sweeps;
  r->rounds0 = st->rounds;
  r->swap_every = swap_every;
  r->dev = dev_state(st);
  int64_t sw = st->sweeps, ro = st->rounds;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    delete r;
    return hip_fail(e, "capture begin");
  }
  rc = enqueue_sweeps(g, r->dev, &sw, &ro, n_sweeps, swap_every, e_series, s);
  e = hipStreamEndCapture(s, &r->graph);
  if (rc) {
    if (r->graph) hipGraphDestroy(r->graph);
    delete r;
    return rc;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&r->exec, r->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (r->graph) hipGraphDestroy(r->graph);
    delete r;
    return hip_fail(e, "capture end / instantiate");
  }
  r->dsweeps = sw - st->sweeps;
  r->drounds = ro - st->rounds;
  *out = r;
  return ISING_OK;
}

extern "C" int32_t ising_replay_launch(ising_replay *r, ising_state *st, void *stream) {
  if (!r || !st) return fail(ISING_E_INVAL, "replay: NULL argument");
  if (st->spins != r->dev.spins || st->mt != r->dev.mt || st->energy != r->dev.energy)
    return fail(ISING_E_STATE, "replay: captured for other state buffers");
  if ((st->rounds & 1) != (r->rounds0 & 1) ||
      (r->swap_every > 0 && st->sweeps % r->swap_every != r->sweeps0 % r->swap_every))
    return fail(ISING_E_STATE, "replay: the state's swap phase differs from the captured one");
  HIP_TRY(hipGraphLaunch(r->exec, (hipStream_t)stream), "replay launch");
  st->sweeps += r->dsweeps;
  st->rounds += r->drounds;
  return ISING_OK;
}

extern "C" void ising_replay_free(ising_replay *r) {
  if (!r) return;
  if (r->exec) hipGraphExecDestroy(r->exec);
  if (r->graph) hipGraphDestroy(r->graph);
  delete r;
}

// ---------------------------------------------------------------------------
// Autotuner: time every admissible launch shape of every bucket on a scratch
// state (single-sweep launches, as in a swap-every-sweep loop) and keep the
// fastest.  The chain does not depend on the shape.
// ---------------------------------------------------------------------------
extern "C" int32_t ising_autotune(ising_graph *g, ising_state *scratch, int32_t reps, void *stream,
                                  int64_t *report, int32_t report_rows) {
  if (!g) return fail(ISING_E_INVAL, "autotune: NULL graph");
  int32_t rc = check_state(scratch);
  if (rc) return rc;
  if (reps < 1) reps = 3;
  hipStream_t s = (hipStream_t)stream;
  DevState d = dev_state(scratch);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "autotune event");
  HIP_TRY(hipEventCreate(&e1), "autotune event");
  int32_t row = 0;
  // When every bucket holds whole ladders, sweeps run in long launches with the
  // swap rounds inside: time launches of 16 sweeps with a round after each,
  // so that the per-sweep cost, not the launch's state load and store, decides.
  const bool ladders = g->ladder_all();
  const int32_t per = ladders ? 16 : 1;
  const LadderArgs la = ladders ? LadderArgs{1, 0, 0, 0} : LadderArgs{0, 0, 0, 0};
  for (size_t bi = 0; bi < g->buckets.size(); ++bi) {
    int32_t Kmax = 1;
    for (int32_t sy : g->bucket_sys[bi]) Kmax = std::max(Kmax, g->sys[sy].K);
    const Bucket orig = g->buckets[bi];
    Bucket best = orig;
    int64_t best_ns = -1;
    for (int32_t tpw = 8; tpw <= 1024; tpw <<= 1) {
      for (int32_t G = 1; G <= 32; G <<= 1) {
        Bucket b = orig;
        if (shape_bucket(b, tpw, G, Kmax, !g->two_field) != ISING_OK || b.G != G) continue;
        if (orig.ladder && !b.ladder) continue;  // keep whole ladders in one workgroup
        g->buckets[bi] = b;
        g->tiles.clear();
        for (size_t i = 0; i < g->buckets.size(); ++i) tile_bucket(*g, g->buckets[i], g->bucket_sys[i]);
        HIP_TRY(hipMemcpyAsync((void *)g->dev.tiles, g->tiles.data(), sizeof(Tile) * g->tiles.size(),
                               hipMemcpyHostToDevice, s),
                "autotune tiles");
        HIP_TRY(launch_sweep(g->dev, d, g->buckets[bi], per, 0, s, la), "autotune warm-up");
        HIP_TRY(hipEventRecord(e0, s), "autotune event");
        for (int32_t k = 0; k < reps; ++k)
          HIP_TRY(launch_sweep(g->dev, d, g->buckets[bi], per, 0, s, la), "autotune trial");
        HIP_TRY(hipEventRecord(e1, s), "autotune event");
        HIP_TRY(hipEventSynchronize(e1), "autotune sync");
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "autotune time");
        const int64_t ns = (int64_t)((double)ms * 1e6 / ((double)reps * per));  // per sweep
        if (report && row < report_rows) {
          int64_t *o = report + (size_t)row * 4;
          o[0] = (int64_t)bi;
          o[1] = tpw;
          o[2] = G;
          o[3] = ns;
          ++row;
        }
        if (best_ns < 0 || ns < best_ns) {
          best_ns = ns;
          best = g->buckets[bi];
        }
      }
    }
    g->buckets[bi] = best;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  g->tiles.clear();
  for (size_t i = 0; i < g->buckets.size(); ++i) tile_bucket(*g, g->buckets[i], g->bucket_sys[i]);
  HIP_TRY(hipMemcpyAsync((void *)g->dev.tiles, g->tiles.data(), sizeof(Tile) * g->tiles.size(),
                         hipMemcpyHostToDevice, s),
          "autotune tiles");
  HIP_TRY(hipStreamSynchronize(s), "autotune sync");
  return row;
}

extern "C" int32_t ising_stats(const ising_graph *g, const ising_state *st, uint64_t *out, void *stream) {
  if (!g || !out) return fail(ISING_E_INVAL, "stats: NULL argument");
  int32_t rc = check_state(st);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_reduce_stats(dev_state(st), (int32_t)g->R, (int32_t)g->slots, s), "stats kernel");
  HIP_TRY(hipMemcpyAsync(out, st->stats, sizeof(uint64_t) * ISING_N_STATS, hipMemcpyDeviceToHost, s), "stats copy");
  HIP_TRY(hipStreamSynchronize(s), "stats sync");
  out[ISING_STAT_ATTEMPTS] = (uint64_t)(st->sweeps > 0 ? st->sweeps : 0) * (uint64_t)g->attempts;
  return ISING_OK;
}

extern "C" int32_t ising_record_slots(const ising_graph *g, const ising_state *st, int32_t *e_row, void *stream) {
  if (!g || !e_row) return fail(ISING_E_INVAL, "record_slots: NULL argument");
  int32_t rc = check_state(st);
  if (rc) return rc;
  HIP_TRY(launch_record(g->dev, dev_state(st), g->n_sys, e_row, (hipStream_t)stream), "record kernel");
  return ISING_OK;
}

extern "C" int32_t pt_swap(const ising_graph *g, ising_state *st, int32_t parity, void *stream) {
  if (!g) return fail(ISING_E_INVAL, "pt_swap: NULL graph");
  int32_t rc = check_state(st);
  if (rc) return rc;
  if (parity != 0 && parity != 1) return fail(ISING_E_INVAL, "pt_swap: parity must be 0 or 1");
  HIP_TRY(launch_swap(g->dev, dev_state(st), g->n_sys, parity, nullptr, (hipStream_t)stream), "swap kernel");
  return ISING_OK;
}

extern "C" int32_t ising_observables(const ising_graph *g, const ising_state *st, int32_t *obs, void *stream) {
  if (!g || !obs) return fail(ISING_E_INVAL, "observables: NULL argument");
  int32_t rc = check_state(st);
  if (rc) return rc;
  HIP_TRY(launch_observables(g->dev, dev_state(st), (int32_t)g->R, obs, 0, (hipStream_t)stream),
          "observables kernel");
  return ISING_OK;
}

extern "C" int32_t ising_refresh_energies(const ising_graph *g, ising_state *st, void *stream) {
  if (!g) return fail(ISING_E_INVAL, "refresh_energies: NULL graph");
  int32_t rc = check_state(st);
  if (rc) return rc;
  HIP_TRY(launch_observables(g->dev, dev_state(st), (int32_t)g->R, nullptr, 1, (hipStream_t)stream),
          "observables kernel");
  return ISING_OK;
}

// ---------------------------------------------------------------------------
// Layer-pair order (Section 3.2, Figure 12c)
// ---------------------------------------------------------------------------
static int32_t check_pairs(const ising_graph *g) {
  if (!g) return fail(ISING_E_INVAL, "layer-pair order: NULL graph");
  if (!g->pair_why.empty()) return fail(ISING_E_RANGE, "layer-pair order: %s", g->pair_why.c_str());
  if (g->two_field) return fail(ISING_E_STATE, "layer-pair order: the two-field form is on");
  return ISING_OK;
}

extern "C" int32_t ising_pairs_words(const ising_graph *g, int64_t *words) {
  int32_t rc = check_pairs(g);
  if (rc) return rc;
  if (!words) return fail(ISING_E_INVAL, "pairs_words: NULL argument");
  *words = (int64_t)kMtN * g->pair_lanes;
  return ISING_OK;
}

extern "C" int32_t ising_pairs_init(const ising_graph *g, ising_state *st, uint32_t *pair_mt,
                                    const uint32_t *pair_seeds, const uint32_t *swap_seeds, void *stream) {
  int32_t rc = check_pairs(g);
  if (rc) return rc;
  rc = check_state(st);
  if (rc) return rc;
  if (!pair_mt || !pair_seeds || !swap_seeds) return fail(ISING_E_INVAL, "pairs_init: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  DevState d = dev_state(st);
  // seeds go to slot 0 of every lane; the seed kernel expands each lane's generator
  HIP_TRY(hipMemcpy2DAsync(pair_mt, 4 * sizeof(uint32_t), pair_seeds, sizeof(uint32_t), sizeof(uint32_t),
                           (size_t)g->pair_lanes, hipMemcpyHostToDevice, s),
          "pairs_init seeds");
  HIP_TRY(hipMemcpy2DAsync(st->swap_mt, kMtN * sizeof(uint32_t), swap_seeds, sizeof(uint32_t), sizeof(uint32_t),
                           (size_t)g->n_sys, hipMemcpyHostToDevice, s),
          "pairs_init swap seeds");
  HIP_TRY(hipStreamSynchronize(s), "pairs_init sync");
  HIP_TRY(launch_pair_seed(pair_mt, g->pair_lanes, s), "pair seed kernel");
  HIP_TRY(launch_seed(d, 0, g->n_sys, s), "swap seed kernel");
  HIP_TRY(hipMemsetAsync(st->flips, 0, sizeof(uint64_t) * g->R, s), "pairs_init clear");
  HIP_TRY(hipMemsetAsync(st->swap_att, 0, sizeof(uint64_t) * g->slots, s), "pairs_init clear");
  HIP_TRY(hipMemsetAsync(st->swap_acc, 0, sizeof(uint64_t) * g->slots, s), "pairs_init clear");
  HIP_TRY(hipMemsetAsync(st->stats, 0, sizeof(uint64_t) * ISING_N_STATS, s), "pairs_init clear");
  HIP_TRY(hipMemsetAsync(st->wsteps, 0, sizeof(uint64_t) * 2 * g->R, s), "pairs_init clear");
  HIP_TRY(launch_labels(g->dev, d, (int32_t)g->R, g->n_sys, s), "labels kernel");
  HIP_TRY(launch_pairs(g->dev, d, pair_mt, g->pair_lanes, g->n_sys, g->pair_threads, g->pair_lds, g->pair_classes,
                       0, 1, LadderArgs{0, 0, 0, 0}, s),
          "initial spins");
  HIP_TRY(launch_observables(g->dev, d, (int32_t)g->R, nullptr, 1, s), "initial energies");
  st->sweeps = 0;
  st->rounds = 0;
  return ISING_OK;
}

extern "C" int32_t ising_pairs_sweep(const ising_graph *g, ising_state *st, uint32_t *pair_mt, int32_t n_sweeps,
                                     int32_t swap_every, void *stream) {
  int32_t rc = check_pairs(g);
  if (rc) return rc;
  rc = check_state(st);
  if (rc) return rc;
  if (!pair_mt) return fail(ISING_E_INVAL, "pairs_sweep: NULL generator array");
  if (n_sweeps < 0 || swap_every < 0) return fail(ISING_E_INVAL, "pairs_sweep: negative count");
  if (st->sweeps < 0) return fail(ISING_E_STATE, "pairs_sweep: state not initialised");
  if (n_sweeps == 0) return ISING_OK;
  const LadderArgs la{swap_every, 0, st->sweeps, st->rounds};
  HIP_TRY(launch_pairs(g->dev, dev_state(st), pair_mt, g->pair_lanes, g->n_sys, g->pair_threads, g->pair_lds,
                       g->pair_classes, n_sweeps, 0, la, (hipStream_t)stream),
          "layer-pair sweep kernel");
  if (swap_every > 0) st->rounds += (st->sweeps + n_sweeps) / swap_every - st->sweeps / swap_every;
  st->sweeps += n_sweeps;
  return ISING_OK;
}

// ---------------------------------------------------------------------------
// Learned cell proposal: network entry points
// ---------------------------------------------------------------------------
static int32_t check_mlp(const ising_mlp *net) {
  if (!net || !net->w || !net->m || !net->v || !net->grad || !net->part || !net->wb)
    return fail(ISING_E_INVAL, "mlp: NULL buffer");
  return ISING_OK;
}

extern "C" int32_t ising_mlp_pack(ising_mlp *net, void *stream) {
  int32_t rc = check_mlp(net);
  if (rc) return rc;
  HIP_TRY(launch_mlp_pack(net->w, net->wb, (hipStream_t)stream), "mlp pack");
  return ISING_OK;
}

extern "C" int32_t ising_mlp_forward(const ising_mlp *net, const float *x, int32_t n, float *logits,
                                     void *stream) {
  int32_t rc = check_mlp(net);
  if (rc) return rc;
  if (n < 0 || (n > 0 && (!x || !logits))) return fail(ISING_E_INVAL, "mlp_forward: bad arguments");
  HIP_TRY(launch_mlp_forward(net->w, net->wb, x, n, logits, (hipStream_t)stream), "mlp forward");
  return ISING_OK;
}

extern "C" int32_t ising_mlp_grad(const ising_mlp *net, const float *x, const uint8_t *y, int32_t n,
                                  float *loss, void *stream) {
  int32_t rc = check_mlp(net);
  if (rc) return rc;
  if (n < 1 || !x || !y) return fail(ISING_E_INVAL, "mlp_grad: bad arguments");
  HIP_TRY(launch_mlp_grad(net->w, net->wb, x, y, n, net->part, net->grad, loss, (hipStream_t)stream), "mlp grad");
  return ISING_OK;
}

extern "C" int32_t ising_mlp_adam(ising_mlp *net, float lr, void *stream) {
  int32_t rc = check_mlp(net);
  if (rc) return rc;
  if (!(lr > 0.f)) return fail(ISING_E_INVAL, "mlp_adam: lr must be > 0");
  net->step += 1;
  HIP_TRY(launch_adam(net->w, net->m, net->v, net->grad, kNParams, lr, 0.9f, 0.999f, 1e-8f, net->step,
                      (hipStream_t)stream),
          "adam");
  HIP_TRY(launch_mlp_pack(net->w, net->wb, (hipStream_t)stream), "mlp pack");
  return ISING_OK;
}

// ---------------------------------------------------------------------------
// Learned cell proposal: cells of the chain
// ---------------------------------------------------------------------------
extern "C" int32_t ising_propose_cells(const ising_graph *g, ising_state *st, const ising_mlp *net, uint64_t key,
                                       int64_t pass_index, uint64_t *moves, void *stream) {
  if (!g) return fail(ISING_E_INVAL, "propose_cells: NULL graph");
  int32_t rc = check_state(st);
  if (rc) return rc;
  rc = check_mlp(net);
  if (rc) return rc;
  if (g->cell_rows == 0) return fail(ISING_E_RANGE, "no system has a grid of 8-spin cells");
  if (g->two_field) return fail(ISING_E_STATE, "cell moves sample the one-field law: turn the two-field form off");
  if (pass_index < 0 || pass_index > (int64_t)UINT32_MAX) return fail(ISING_E_RANGE, "pass_index must fit 32 bits");
  hipStream_t s = (hipStream_t)stream;
  const DevState d = dev_state(st);
  for (int32_t p = 0; p < g->max_phases; ++p)
    HIP_TRY(launch_cell_propose(g->dev, d, g->n_sys, g->cell_rows, p, net->w, net->wb, key, pass_index, moves, s),
            "cell moves");
  return ISING_OK;
}

extern "C" int32_t ising_heatbath_cells(const ising_graph *g, ising_state *st, uint64_t key, int64_t pass_index,
                                        uint64_t *moves, void *stream) {
  if (!g) return fail(ISING_E_INVAL, "heatbath_cells: NULL graph");
  int32_t rc = check_state(st);
  if (rc) return rc;
  if (g->cell_rows == 0) return fail(ISING_E_RANGE, "no system has a grid of 8-spin cells");
  if (g->two_field) return fail(ISING_E_STATE, "cell moves sample the one-field law: turn the two-field form off");
  if (pass_index < 0 || pass_index > (int64_t)UINT32_MAX) return fail(ISING_E_RANGE, "pass_index must fit 32 bits");
  const DevState d = dev_state(st);
  for (int32_t p = 0; p < g->max_phases; ++p)
    HIP_TRY(launch_cell_heatbath(g->dev, d, g->cell_rows, p, key, pass_index, moves, (hipStream_t)stream),
            "heat-bath cell moves");
  return ISING_OK;
}

extern "C" int32_t ising_collect_cells(const ising_graph *g, const ising_state *st, int64_t stride,
                                       int64_t offset, int32_t n, float *x, uint8_t *y, void *stream) {
  if (!g || !x || !y || n < 0 || stride < 1 || offset < 0) return fail(ISING_E_INVAL, "collect_cells: bad arguments");
  int32_t rc = check_state(st);
  if (rc) return rc;
  if (g->total_cells == 0) return fail(ISING_E_RANGE, "no system has a grid of 8-spin cells");
  HIP_TRY(launch_collect_cells(g->dev, dev_state(st), g->n_sys, stride, offset, g->total_cells, n, x, y,
                               (hipStream_t)stream),
          "collect cells");
  return ISING_OK;
}
