// Host-only part of libising: validation and packing of the systems, the
// launch plan (buckets, shapes, tiles), the threshold rows and the error
// message of the C ABI.  It uses no HIP runtime call, so it also builds with a
// plain C++ compiler (the sanitizer build of the tests does that).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ising.h"
#include "internal.h"

namespace ising {

// Record the message of a failing call (thread-local, ising_last_error) and
// return `code`.
int32_t fail(int32_t code, const char *fmt, ...);

struct SysHost {
  int32_t S, M, ring, F, deg, dmax, K, cell, FW;
  int32_t ds = 0, dt = 0;  // two-field bounds: max |h| + sum |J in-slice|, max sum |J_tau| of a spin
  int32_t grid_L = 0, n_phases = 0;
  int32_t cell_fast = 0;  // cell records carry couplings by direction (every outside neighbour of spin k is spin k)
  std::vector<uint16_t> cells;  // cell indices, phase by phase
  int32_t pc[5] = {0, 0, 0, 0, 0};
  std::vector<TmplSpin> tmpl;
  std::vector<uint32_t> fifo;  // (queue base << 8) | log2(depth) per template spin
  std::vector<uint16_t> lanes;  // sweep lane position -> template spin, by level offset
  std::vector<uint32_t> cellrec;  // grid templates: kCellRecWords words per template cell
  std::vector<double> beta;
};

// Validate one system description and pack its template (rows with J inline,
// schedule offsets, uniform queues, cell records).
int32_t build_system(const ising_system_desc &d, int32_t idx, SysHost &out);
int32_t build_all(const ising_system_desc *sys, int32_t n_sys, std::vector<SysHost> &hs);

// Everything about a loaded graph that the host decides: per-system records,
// buckets, launch shapes and tiles, per-slot beta, the two-field bounds and
// the layer-pair launch.  The library's graph handle adds the device side.
struct GraphPlan {
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
  std::vector<int32_t> slot_dmax;  // largest |h| + sum |J| of the slot's system (the rows' last entry read)
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
  // Streams of a sweep with several buckets.  HIP maps a process's streams onto
  // a few hardware queues (GPU_MAX_HW_QUEUES, 4 by default), and the kernels of
  // one queue run one after another, so a sweep uses at most that many streams
  // (stream 0 is the caller's): bucket b runs on stream_of[b], the buckets are
  // enqueued in launch_order (largest cost first), and the buckets are spread
  // over the streams largest first onto the least loaded one.  bucket_cost[b]
  // is the bucket's time per sweep as the autotuner measured it, else its
  // attempts per sweep.
  std::vector<int64_t> bucket_cost;
  std::vector<int32_t> stream_of, launch_order;
  int32_t n_streams = 1;
  // LDS words of a walker slot for system s in the current form
  int32_t walker_words(int32_t s) const {
    const SysInfo &si = sys[s];
    return two_field ? walker_lds_words(si.S, si.WW, si.fifo_words, si.RS, std::max(qrow, kThrRow), 5)
                     : walker_lds_words(si.S, si.WW, si.fifo_words, si.RS);
  }
};

// Byte offsets of the device tables in the caller's buffer.
struct Layout {
  size_t sys, tmpl, fifo, lanes, thr, beta, tiles, wsys, cells, rtiles, cellrec, qthr, qa, qc, total;
};
Layout layout_for(int64_t n_sys, int64_t n_tmpl, int64_t slots, int64_t n_tiles, int64_t R, int64_t n_cells,
                  int64_t cell_rows, int64_t n_cellrec, int64_t qrow);

// Launch shape of a bucket (ISING_E_RANGE when it does not fit) and the
// default shape of a template size.
int32_t shape_bucket(Bucket &b, int32_t tpw, int32_t G, int32_t Kmax, bool allow_ladder = true);
void default_shape(int32_t S, int32_t walker_words, int32_t Kmax, int32_t &tpw, int32_t &G, bool allow_ladder = true);
// Threads per walker the autotuner tries for a template of S spins: the powers
// of two from 8 to 1024, and above 64 the counts that leave few idle lanes:
// S and ceil(S / 2) (one or two columns per thread, walkers back to back) and
// their multiples of 64.
std::vector<int32_t> tpw_candidates(int32_t S);
// Tiles of a bucket appended to g.tiles; all buckets' tiles rebuilt in order.
void tile_bucket(GraphPlan &g, Bucket &b, const std::vector<int32_t> &systems);
void retile(GraphPlan &g);
// Systems, slots, buckets and default shapes of a batch of packed systems.
int32_t plan(const std::vector<SysHost> &hs, GraphPlan &g);
// Spread the buckets over at most max_streams streams by their bucket_cost
// (largest first, each onto the stream with the least cost so far).
void assign_streams(GraphPlan &g, int32_t max_streams);
// Hardware queues a process gets (GPU_MAX_HW_QUEUES, else HIP's default of 4; 1..8).
int32_t hw_queues();

// Most sweeps one launch of the sweep kernel (bucket b, its current shape) may
// run: its per-launch 32-bit counters (flips, wavefront steps and steps with a
// flip of a walker, swap acceptances of a pair, and a lane's sum of d over its
// flips) then cannot wrap.  The graph's limit is the smallest over its buckets.
int64_t bucket_sweep_limit(const GraphPlan &g, size_t b);
int64_t sweep_limit(const GraphPlan &g);
// The same for the layer-pair kernel (flips of a walker, a lane's sum of d).
int64_t pairs_sweep_limit(const GraphPlan &g);
// A lower cap from the environment (ISING_LAUNCH_SWEEPS_MAX, when set to n >= 1):
// calls then run as launches of at most n sweeps, which lets a test drive the
// cut into segments without running 10^5 sweeps.
int64_t launch_sweeps_cap();

}  // namespace ising
