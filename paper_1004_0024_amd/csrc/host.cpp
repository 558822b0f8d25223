// Host-only part of libising (see host.h): validation and packing of the
// systems into device tables, launch planning, threshold rows.
#include "host.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

using namespace ising;

static thread_local std::string g_err;

namespace ising {
int32_t fail(int32_t code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
}  // namespace ising

extern "C" const char *ising_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// Host-only helpers
// ---------------------------------------------------------------------------
extern "C" int32_t ising_threshold_row(double beta, int32_t dmax, uint32_t *thr) {
  if (!thr || dmax < 0 || dmax > 1023) return fail(ISING_E_INVAL, "threshold_row: bad arguments");
  if (!(beta > 0.0) || !isfinite(beta)) return fail(ISING_E_RANGE, "threshold_row: beta must be > 0");
  // exp(-2 beta d) must stay a normal double: once it underflows to 0 the
  // threshold ceil(2^32 p) - 1 would wrap to all ones (always flip) where the
  // rule never flips
  if (2.0 * beta * (double)dmax > 700.0)
    return fail(ISING_E_RANGE, "threshold_row: 2 beta d_max = %g exceeds 700", 2.0 * beta * (double)dmax);
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

namespace ising {

int32_t build_system(const ising_system_desc &d, int32_t idx, SysHost &out) {
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
  for (int32_t k = 0; k < d.n_temps; ++k)  // the threshold rows' range (ising_threshold_row)
    if (2.0 * d.beta[k] * (double)out.dmax > 700.0)
      return fail(ISING_E_RANGE, "system %d: 2 beta[%d] d_max = %g exceeds 700", idx, k,
                  2.0 * d.beta[k] * (double)out.dmax);
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
      out.cell_fast = 1;
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
            if ((nb & 7) != k) out.cell_fast = 0;
            rec[24 + k] |= (uint32_t)(uint8_t)(int8_t)(2 * t.J[j]) << (8 * dir);
          }
          rec[16 + (k >> 2)] |= (uint32_t)(uint8_t)t.h << (8 * (k & 3));
          rec[18 + (k >> 2)] |= (uint32_t)(uint8_t)t.Jtau << (8 * (k & 3));
          if (k < 4) rec[20 + k] = (uint32_t)t.jpack;
          int32_t hc = t.h - 2 * t.Jtau;  // the field's constant part with s = 2 bit - 1
          for (int32_t j = 4; j < t.deg; ++j) hc -= t.J[j];
          if (hc < -128 || hc > 127) out.cell_fast = 0;
          rec[32 + (k >> 2)] |= (uint32_t)(uint8_t)(int8_t)hc << (8 * (k & 3));
          if (k < 4) {  // minus the sum of J from spin k to spins 4..7 of the cell, int16
            int32_t js = 0;
            for (int32_t i = 0; i < 4; ++i) js += (int32_t)(int8_t)((uint32_t)t.jpack >> (8 * i)) / 2;
            rec[34 + (k >> 1)] |= (uint32_t)(uint16_t)(int16_t)(-js) << (16 * (k & 1));
          }
        }
      }
    }
  }
  out.beta.assign(d.beta, d.beta + d.n_temps);
  return ISING_OK;
}


}  // namespace ising

extern "C" int32_t ising_level_offsets(const ising_system_desc *sys, int32_t *f, int32_t *depth) {
  if (!sys || !f || !depth) return fail(ISING_E_INVAL, "level_offsets: NULL argument");
  SysHost h;
  int32_t rc = build_system(*sys, 0, h);
  if (rc) return rc;
  for (int32_t q = 0; q < h.S; ++q) f[q] = h.tmpl[q].f;
  *depth = h.F;
  return ISING_OK;
}

namespace ising {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device tables.  Room for one tile per walker, so any launch shape can be
// installed later without reallocating.
Layout layout_for(int64_t n_sys, int64_t n_tmpl, int64_t slots, int64_t n_tiles, int64_t R, int64_t n_cells,
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
  o = align256(o + sizeof(uint32_t) * std::max<int64_t>(n_cells, 1));
  L.rtiles = o;
  o = align256(o + 2 * sizeof(int32_t) * std::max<int64_t>(cell_rows / 64, 1));
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

// Launch shape of a bucket: `tpw` threads per walker (a power of two up to 64,
// a multiple of 64 up to 1024, or another count from 65 to 1024 when that
// leaves at most two columns per thread; each thread owns ceil(S/tpw) <= 8
// columns) and G walkers per workgroup.
int32_t shape_bucket(Bucket &b, int32_t tpw, int32_t G, int32_t Kmax, bool allow_ladder) {
  if (tpw < 1 || tpw > 1024 || (tpw <= 64 && (tpw & (tpw - 1)) != 0))
    return fail(ISING_E_RANGE, "tpw must be a power of two up to 64, or 65..1024");
  const int32_t need = (b.S + tpw - 1) / tpw;
  int32_t cpt = 1;
  while (cpt < need) cpt <<= 1;
  if (cpt > 8) return fail(ISING_E_RANGE, "tpw=%d leaves %d columns per thread (max 8)", tpw, need);
  if (tpw > 64 && tpw % 64 != 0 && cpt > 2)
    return fail(ISING_E_RANGE, "tpw=%d (not a multiple of 64) leaves %d columns per thread (max 2)", tpw, need);
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
void default_shape(int32_t S, int32_t walker_words, int32_t Kmax, int32_t &tpw, int32_t &G, bool allow_ladder) {
  int32_t p = 8;
  while (p < S) p <<= 1;
  tpw = p >= 256 ? p / 2 : p;
  G = std::max(1, 256 / tpw);
  while (G > 1 && (size_t)G * walker_words * 4 > 40 * 1024) --G;
  if (allow_ladder && G < Kmax && tpw <= 64 && (int64_t)Kmax * tpw <= 1024 &&
      ((size_t)Kmax * walker_words + kLadderWords) * 4 <= 160 * 1024)
    G = Kmax;
}

void tile_bucket(GraphPlan &g, Bucket &b, const std::vector<int32_t> &systems) {
  b.tile0 = (int32_t)g.tiles.size();
  for (int32_t s : systems)
    for (int32_t w0 = 0; w0 < g.sys[s].K; w0 += b.G)
      g.tiles.push_back(Tile{s, w0, std::min(b.G, g.sys[s].K - w0), 0});
  b.ntiles = (int32_t)g.tiles.size() - b.tile0;
}

std::vector<int32_t> tpw_candidates(int32_t S) {
  std::vector<int32_t> v;
  for (int32_t t = 8; t <= 1024; t <<= 1) v.push_back(t);
  for (int32_t t : {S, (S + 1) / 2})
    if (t > 64 && t <= 1024) {
      v.push_back(t);
      v.push_back(std::min(1024, (t + 63) / 64 * 64));
    }
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  return v;
}

void retile(GraphPlan &g) {
  g.tiles.clear();
  for (size_t i = 0; i < g.buckets.size(); ++i) tile_bucket(g, g.buckets[i], g.bucket_sys[i]);
}

int32_t plan(const std::vector<SysHost> &hs, GraphPlan &g) {
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
    si.cell_fast = h.cell_fast;
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
    int64_t attempts = 0;
    for (int32_t s : kv.second) attempts += (int64_t)g.sys[s].K * g.sys[s].S * g.sys[s].M;
    g.buckets.push_back(b);
    g.bucket_sys.push_back(kv.second);
    g.bucket_cost.push_back(attempts);
  }
  assign_streams(g, hw_queues());
  return ISING_OK;
}

void assign_streams(GraphPlan &g, int32_t max_streams) {
  const int32_t nb = (int32_t)g.buckets.size();
  g.n_streams = std::max(1, std::min(nb, max_streams));
  g.launch_order.resize(nb);
  for (int32_t b = 0; b < nb; ++b) g.launch_order[b] = b;
  std::stable_sort(g.launch_order.begin(), g.launch_order.end(),
                   [&](int32_t a, int32_t b) { return g.bucket_cost[a] > g.bucket_cost[b]; });
  std::vector<int64_t> load(g.n_streams, 0);
  g.stream_of.assign(nb, 0);
  for (int32_t b : g.launch_order) {
    int32_t best = 0;
    for (int32_t q = 1; q < g.n_streams; ++q)
      if (load[q] < load[best]) best = q;
    g.stream_of[b] = best;
    load[best] += g.bucket_cost[b];
  }
}

int32_t hw_queues() {
  const char *v = getenv("GPU_MAX_HW_QUEUES");
  int32_t n = v ? atoi(v) : 4;
  return n < 1 ? 4 : (n > 8 ? 8 : n);
}

int32_t build_all(const ising_system_desc *sys, int32_t n_sys, std::vector<SysHost> &hs) {
  if (!sys || n_sys < 1) return fail(ISING_E_INVAL, "need at least one system");
  hs.resize(n_sys);
  for (int32_t s = 0; s < n_sys; ++s) {
    int32_t rc = build_system(sys[s], s, hs[s]);
    if (rc) return rc;
  }
  return ISING_OK;
}


// Per sweep, a walker of system s in bucket b adds at most: N = S M flips;
// (ceil(tpw / 64) + 1) wavefronts x cpt columns x (M + F - 1) levels wavefront
// steps (a wavefront's steps go to the walker of its first lane, and the
// wavefronts whose first lane is one of a walker's are at most that many; when
// tpw < 64 that walker takes the steps of the wavefront's other walkers too, at
// most one per column slot and level); and a lane's |2 sum d| grows by at most
// 2 * 63 * cpt * M.  A pair's acceptances grow by at most one per sweep.
int64_t bucket_sweep_limit(const GraphPlan &g, size_t b) {
  const Bucket &bk = g.buckets[b];
  int64_t lim = INT32_MAX;  // n_sweeps is an int32
  for (int32_t s : g.bucket_sys[b]) {
    const SysInfo &si = g.sys[s];
    const int64_t N = (int64_t)si.S * si.M;
    const int64_t waves = (bk.tpw + 63) / 64 + 1;
    const int64_t steps = waves * bk.cpt * (int64_t)(si.M + si.F - 1);
    const int64_t dsum = 2 * 63 * (int64_t)bk.cpt * si.M;
    lim = std::min(lim, (int64_t)UINT32_MAX / std::max(N, steps));
    lim = std::min(lim, (int64_t)INT32_MAX / dsum);
  }
  return std::max<int64_t>(lim, 1);
}

int64_t sweep_limit(const GraphPlan &g) {
  int64_t lim = INT32_MAX;
  for (size_t b = 0; b < g.buckets.size(); ++b) lim = std::min(lim, bucket_sweep_limit(g, b));
  return std::min(lim, launch_sweeps_cap());
}

int64_t launch_sweeps_cap() {
  const char *v = getenv("ISING_LAUNCH_SWEEPS_MAX");
  const long long n = v ? atoll(v) : 0;
  return n >= 1 ? (int64_t)n : INT32_MAX;
}

// Layer-pair kernel: a walker flips at most N spins per sweep, and a lane (two
// slices of S spins) changes |2 sum d| by at most 2 * 63 * 2 S.
int64_t pairs_sweep_limit(const GraphPlan &g) {
  int64_t lim = INT32_MAX;
  for (const SysInfo &si : g.sys) {
    lim = std::min(lim, (int64_t)UINT32_MAX / ((int64_t)si.S * si.M));
    lim = std::min(lim, (int64_t)INT32_MAX / (2 * 63 * 2 * (int64_t)si.S));
  }
  return std::max<int64_t>(std::min(lim, launch_sweeps_cap()), 1);
}

}  // namespace ising

extern "C" int32_t ising_graph_bytes(const ising_system_desc *sys, int32_t n_sys, size_t *dev_bytes) {
  if (!dev_bytes) return fail(ISING_E_INVAL, "dev_bytes is NULL");
  std::vector<SysHost> hs;
  int32_t rc = build_all(sys, n_sys, hs);
  if (rc) return rc;
  GraphPlan g;
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
