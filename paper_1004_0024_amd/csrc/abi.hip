// Device side of the C ABI declared in include/ising.h: loading the packed
// tables, the chain's state, launch sequencing, captured loops and the
// autotuner.  Validation and planning are in host.cpp.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/ising.h"
#include "host.h"
#include "internal.h"
#include "mlp.h"

using namespace ising;

static int32_t hip_fail(hipError_t e, const char *where) {
  return fail(ISING_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(expr, where)                     \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// ---------------------------------------------------------------------------
// Graph handle
// ---------------------------------------------------------------------------
struct ising_graph : GraphPlan {
  DevTables dev{};
  size_t bytes = 0;
  // With several buckets, stream q > 0 of the plan (stream_of) is side[q - 1],
  // forked from and joined back to the caller's stream, so the buckets of one
  // sweep run side by side and each one's tail overlaps the others.
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;  // ev[0]: fork; ev[q]: stream q done
  ~ising_graph() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipStream_t q : side) (void)hipStreamDestroy(q);
  }
};

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
        // entries d = 1 .. d_max of the system; larger d never occur there
        uint32_t row[kThrRow - kThrZero] = {0};
        rc = ising_threshold_row(h.beta[k], h.dmax, row);
        if (rc) {
          delete g;
          return rc;
        }
        for (int32_t i = 0; i < kThrRow; ++i) thr[i] = i <= kThrZero ? 0xffffffffu : row[i - kThrZero];
        thr += kThrRow;
        *bt++ = h.beta[k];
        g->slot_beta.push_back(h.beta[k]);
        g->slot_dmax.push_back(h.dmax);
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
  {  // cell lists: index (m*L + y)*L + x -> (m << 16) | (y << 8) | x (L <= 255 for a grid)
    uint32_t *co = (uint32_t *)(host.data() + L.cells);
    for (size_t i = 0; i < hs.size(); ++i) {
      const uint32_t gl = (uint32_t)std::max(g->sys[i].grid_L, 1);
      for (uint16_t c : hs[i].cells) {
        const uint32_t m = c / (gl * gl), y = (c / gl) % gl, x = c % gl;
        *co++ = (m << 16) | (y << 8) | x;
      }
    }
  }
  {
    uint32_t *cr = (uint32_t *)(host.data() + L.cellrec);
    for (auto &h : hs) {
      memcpy(cr, h.cellrec.data(), sizeof(uint32_t) * h.cellrec.size());
      cr += h.cellrec.size();
    }
  }
  {  // each 64-row tile of cell moves: the last system whose rows start at or before it, and
     // the walker of its first row (K for a tile of padding rows)
    int32_t *ts = (int32_t *)(host.data() + L.rtiles);
    int32_t sidx = 0;
    for (int64_t t = 0; t < g->cell_rows / 64; ++t) {
      while (sidx + 1 < n_sys && g->sys[sidx + 1].row0 <= t * 64) ++sidx;
      const SysInfo &si = g->sys[sidx];
      ts[2 * t] = sidx;
      ts[2 * t + 1] = si.rows > 0 ? (int32_t)std::min<int64_t>((t * 64 - si.row0) / si.rows, si.K) : si.K;
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
  g->dev.cells = (const uint32_t *)(base + L.cells);
  g->dev.cell_tiles = (const int2 *)(base + L.rtiles);
  g->dev.cellrec = (const uint32_t *)(base + L.cellrec);
  g->dev.qthr = (const uint32_t *)(base + L.qthr);
  g->dev.qa = (const double *)(base + L.qa);
  g->dev.qc = (const double *)(base + L.qc);
  g->dev.two_field = 0;
  g->dev.qrow = g->qrow;
  g->dev.qwt = 2 * g->qdt + 1;
  g->dev.qoff = g->qds * (2 * g->qdt + 1) + g->qdt;
  g->bytes = L.total;
  if (g->n_streams > 1) {
    for (int32_t b = 0; b < g->n_streams; ++b) {
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
    uint32_t row[kThrRow - kThrZero] = {0};
    const int32_t rc = ising_acceptance_row(g->slot_beta[k], g->slot_dmax[k], kind, row);
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
  retile(*g);
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
  const int64_t v[13] = {b.S, (int64_t)g->bucket_sys[bucket].size(), walkers, attempts, b.tpw, b.G,
                         b.cpt, b.threads, (int64_t)b.lds, b.ntiles, b.ladder, g->stream_of[bucket],
                         g->bucket_cost[bucket]};
  for (int32_t i = 0; i < n && i < 13; ++i) out[i] = v[i];
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
  retile(*g);
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
  c[12] = g->slots;
  return ISING_OK;
}

static int32_t check_state(const ising_state *st) {
  if (!st || !st->spins || !st->mt || !st->energy || !st->temp_of || !st->walker_at || !st->swap_mt ||
      !st->flips || !st->swap_att || !st->swap_acc || !st->stats || !st->wsteps || !st->bond ||
      !st->swap_near)
    return fail(ISING_E_INVAL, "state has a NULL buffer");
  return ISING_OK;
}

static DevState dev_state(const ising_state *st) {
  return DevState{st->spins, st->mt, st->energy, st->temp_of, st->walker_at, st->swap_mt,
                  st->flips, st->swap_att, st->swap_acc, st->stats, st->wsteps, st->bond, st->swap_near};
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
  HIP_TRY(hipMemsetAsync(st->swap_near, 0, sizeof(uint64_t) * g->slots, s), "init_state clear");
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
// Launch every bucket, largest first: on the caller's stream s, or with several
// streams each bucket on its stream of the plan (side streams forked from and
// joined back to s).
static int32_t launch_buckets(const ising_graph *g, const DevState &d, int32_t n, LadderArgs la, hipStream_t s) {
  if (g->side.empty()) {
    for (int32_t b : g->launch_order) HIP_TRY(launch_sweep(g->dev, d, g->buckets[b], n, 0, s, la), "sweep kernel");
    return ISING_OK;
  }
  HIP_TRY(hipEventRecord(g->ev[0], s), "fork");
  for (size_t q = 0; q < g->side.size(); ++q) HIP_TRY(hipStreamWaitEvent(g->side[q], g->ev[0], 0), "fork wait");
  for (int32_t b : g->launch_order) {
    const int32_t q = g->stream_of[b];
    HIP_TRY(launch_sweep(g->dev, d, g->buckets[b], n, 0, q == 0 ? s : g->side[q - 1], la), "sweep kernel");
  }
  for (size_t q = 0; q < g->side.size(); ++q) {
    HIP_TRY(hipEventRecord(g->ev[q + 1], g->side[q]), "join record");
    HIP_TRY(hipStreamWaitEvent(s, g->ev[q + 1], 0), "join");
  }
  return ISING_OK;
}

// A launch runs at most sweep_limit(*g) sweeps, so that its 32-bit counters
// cannot wrap; longer calls are cut into launches of at most that many.
static int32_t enqueue_sweeps(const ising_graph *g, const DevState &d, int64_t *sweeps, int64_t *rounds,
                              int32_t n_sweeps, int32_t swap_every, int32_t *e_series, hipStream_t s) {
  const int64_t lim = sweep_limit(*g);
  if (swap_every > 0 && !e_series && n_sweeps > 0 && g->ladder_all()) {
    // every system's ladder sits in one workgroup: sweeps and swap rounds in one launch
    for (int32_t done = 0; done < n_sweeps;) {
      const int32_t seg = (int32_t)std::min<int64_t>(n_sweeps - done, lim);
      const LadderArgs la{swap_every, 0, *sweeps, *rounds};
      int32_t rc = launch_buckets(g, d, seg, la, s);
      if (rc) return rc;
      *rounds += (*sweeps + seg) / swap_every - *sweeps / swap_every;
      *sweeps += seg;
      done += seg;
    }
    return ISING_OK;
  }
  int32_t done = 0;
  while (done < n_sweeps) {
    // Sweeps until the next swap round (or the end, or the next record).
    int32_t seg = (int32_t)std::min<int64_t>(n_sweeps - done, lim);
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
// Autotuner: time every admissible launch shape of every bucket (threads per
// walker from tpw_candidates, 1 to 32 walkers per workgroup) on a scratch
// state (single-sweep launches, as in a swap-every-sweep loop) and keep the
// fastest; the kept shapes' times then spread the buckets over the streams.
// The chain does not depend on the shape.
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
    for (int32_t tpw : tpw_candidates(orig.S)) {
      for (int32_t G = 1; G <= 32; G <<= 1) {
        Bucket b = orig;
        if (shape_bucket(b, tpw, G, Kmax, !g->two_field) != ISING_OK || b.G != G) continue;
        if (orig.ladder && !b.ladder) continue;  // keep whole ladders in one workgroup
        g->buckets[bi] = b;
        retile(*g);
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
    if (best_ns > 0) g->bucket_cost[bi] = best_ns;  // the bucket's own time per sweep
  }
  // spread the buckets over the streams by their measured times
  assign_streams(*g, (int32_t)g->side.size() + 1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  retile(*g);
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
  HIP_TRY(hipMemsetAsync(st->swap_near, 0, sizeof(uint64_t) * g->slots, s), "pairs_init clear");
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
  // launches of at most pairs_sweep_limit sweeps: their 32-bit counters cannot wrap
  const int64_t lim = pairs_sweep_limit(*g);
  for (int32_t done = 0; done < n_sweeps;) {
    const int32_t seg = (int32_t)std::min<int64_t>(n_sweeps - done, lim);
    const LadderArgs la{swap_every, 0, st->sweeps, st->rounds};
    HIP_TRY(launch_pairs(g->dev, dev_state(st), pair_mt, g->pair_lanes, g->n_sys, g->pair_threads, g->pair_lds,
                         g->pair_classes, seg, 0, la, (hipStream_t)stream),
            "layer-pair sweep kernel");
    if (swap_every > 0) st->rounds += (st->sweeps + seg) / swap_every - st->sweeps / swap_every;
    st->sweeps += seg;
    done += seg;
  }
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

extern "C" int32_t ising_mlp_grad_noalloc(const ising_mlp *net, const float *x, const uint8_t *y, int32_t n,
                                          float *loss, void *stream) {
  if (!net || !net->w || !net->grad || !net->wb) return fail(ISING_E_INVAL, "mlp_grad_noalloc: NULL buffer");
  if (n < 1 || !x || !y) return fail(ISING_E_INVAL, "mlp_grad_noalloc: bad arguments");
  if (mlp_grad_parts(n) > ISING_MLP_PARTS)
    return fail(ISING_E_SIZE, "mlp_grad_noalloc: %d partial gradients exceed the %d rows of the library's scratch",
                mlp_grad_parts(n), ISING_MLP_PARTS);
  float *rows = nullptr;
  HIP_TRY(mlp_scratch_rows(&rows), "mlp_grad_noalloc: scratch address");
  HIP_TRY(launch_mlp_grad(net->w, net->wb, x, y, n, rows, net->grad, loss, (hipStream_t)stream), "mlp grad");
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
