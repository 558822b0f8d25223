// Internal layout shared by the host side and the kernels of libising.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

namespace ising {

constexpr int kMtN = 624;       // MT19937 words
constexpr int kMtM = 397;       // MT19937 middle offset
constexpr int kMtLag = 227;     // kMtN - kMtM: words generated without a chain
// Threshold row of a temperature slot on the device: entry kThrZero + d for
// d = -64..63 (every entry with d <= 0 is 0xffffffff: such a flip always
// passes), so the sweep indexes it with d directly.
constexpr int kThrRow = 128;
constexpr int kThrZero = 64;
constexpr int kPairThrRow = 64;  // the layer-pair kernel keeps entries d = 0..63 of the row
constexpr int kMaxDeg = 8;      // in-slice neighbours in a template record

// One system, as the kernels see it.
struct SysInfo {
  int32_t S, M, ring, F;   // spins per slice, slices, ring flag, schedule depth
  int32_t RS, WW;          // words per slice row (odd when > 1: no LDS bank aliasing), per walker
  int32_t K, walker0;      // walkers (= slots), global index of walker 0
  int64_t spin_word0;      // first spin word of walker 0
  int32_t tmpl0;           // first template record
  int32_t thr0;            // first threshold row (K rows of kThrRow words)
  int32_t slot0;           // first global slot
  int32_t deg;             // max in-slice degree of the template
  int32_t cell;            // 1: every spin's first 4 neighbours are the other half of its 8-spin cell
  int32_t nx;              // neighbours handled one by one (deg, or deg - 4 for cell templates)
  int32_t fifo_words;      // per walker: LDS words of the uniform queues
  int32_t cb0;             // first cell record (kCellRecWords words each) of the template's cells
  // cell moves (learned proposal); grid_L = 0 when the template is not a grid of 8-spin cells
  int32_t grid_L;          // cells per grid side: cell (m, y, x) = spins m*S + (y*L + x)*8 + 0..7
  int32_t n_phases;        // colour classes of cells (2, or 4 on a ring of odd length)
  int32_t cl0;             // first entry of this system's cell list
  int32_t pc[5];           // phase p owns cell-list entries [pc[p], pc[p+1])
  int32_t rows;            // proposal work rows per walker (largest phase)
  int32_t pl0;             // layer-pair order: first generator lane of walker 0 (M/2 per walker)
  int32_t cell_fast;       // 1: every outside in-slice neighbour of cell spin k is spin k of its cell
                           // (K4,4 grids): cell records then carry couplings by direction
  int64_t row0;            // first proposal work row of walker 0
  int64_t cell0;           // global index of walker 0's cell 0 (cells numbered walker-major)
};

// Template spin q: in-slice neighbours with their couplings, field, tau coupling,
// level offset.  Unused neighbour entries point at q itself with J = 0.  For a
// cell template nbr[0..3] are the partners q' = (q & ~7) + ((q & 4) ^ 4) + i and
// jpack holds their 2J as four signed bytes (byte i for partner i).
struct TmplSpin {
  int16_t nbr[kMaxDeg];
  int8_t J[kMaxDeg];
  int8_t h, Jtau;
  uint8_t f, deg;
  int32_t jpack;
};
static_assert(sizeof(TmplSpin) == 32, "template record is 32 bytes");

// Cell record of a template cell c (cell moves), kCellRecWords uint32 words:
//   [2k], [2k+1]  spin k's in-slice neighbours outside the cell, four 16-bit
//                 entries: low byte J (int8, 0 for an unused entry), bits 8..12
//                 the bit of that neighbour in the word (cell byte above) | (below
//                 << 8) | (left << 16) | (right << 24);
//   [16], [17]    h_k as int8, k = 0..3 and 4..7;
//   [18], [19]    J_tau of spin k as int8;
//   [20 + k]      2J of spin k (< 4) to the spins 4 + i of the cell, byte i;
//   [24 + k]      when the system's cell_fast is set: 2J of spin k to spin k of
//                 the cell above, below, left and right, bytes 0..3 (0 where
//                 there is none), matching the byte order of the word above;
//   [32], [33]    when cell_fast is set: h_k - sum_dir J - 2 J_tau as int8,
//                 k = 0..3 and 4..7 (the constant part of the boundary field when
//                 bits stand for spins: s = 2 bit - 1);
//   [34], [35]    minus the sum over i of J between spin k < 4 and spin 4 + i,
//                 int16, k = 0, 1 and 2, 3.
constexpr int kCellRecWords = 40;

// One workgroup of the sweep: `nw` walkers of system `sys` starting at `w0`.
struct Tile {
  int32_t sys, w0, nw, pad;
};

// Launch geometry of one bucket of tiles (systems with the same S and kernel variant).
struct Bucket {
  int32_t S, G, tpw, cpt;   // template size, walkers per tile, threads per walker, columns per thread
  int32_t ring, nx, cell;   // kernel variant
  int32_t tile0, ntiles;    // tiles [tile0, tile0 + ntiles)
  int32_t threads;          // workgroup size
  int32_t walker_words;     // LDS words per walker slot (max over the bucket's systems)
  int32_t kmax;             // most walkers of a system in the bucket
  int32_t ladder;           // 1: every tile holds a whole system (swap rounds can run in the kernel)
  size_t lds;               // dynamic LDS bytes
};

// In-kernel swap rounds of a ladder bucket: after sweep t of the launch,
// a round runs when (sweeps0 + t + 1) is a multiple of swap_every (0: none);
// round n of the launch uses parity (rounds0 + n) mod 2.
struct LadderArgs {
  int32_t swap_every, pad;
  int64_t sweeps0, rounds0;
};
// LDS words after the walker slots of a ladder workgroup: the swap stream's
// 624-word window, walker at each slot, slot of each walker, the window's head
// (and 3 spare words), accepted swaps per slot, and the outcome of each pair of
// the last round.
constexpr int kLadderWords = kMtN + 256 + 256 + 4 + 256 + 128;

// Generator ring: the 624-word look-back of MT19937 plus one chunk of S words,
// rounded up to whole chunks.  A kMtN-word copy of its top slots sits in front
// of slot 0, so look-back reads never wrap.
__host__ __device__ inline int32_t gen_ring_words(int32_t S) { return S * (1 + (kMtN + S - 1) / S); }

// Uniform queue of template spin q: the uniforms of its column wait there from
// generation (one level before the slice starts) until its visit f(q) levels
// later; f(q) + 2 slots, rounded up to a power of two.
__host__ __device__ inline int32_t fifo_depth(int32_t f) {
  int32_t d = 2;
  while (d < f + 2) d <<= 1;
  return d;
}

// LDS words of one walker slot: generator ring (+ shadow), uniform queues,
// spins (M rows of RS words, with one halo row before and one after), threshold
// row, reduction slots (running cost, flips, wavefront steps, steps with a
// flip; in the two-field form also the running tau-bond sum).
__host__ __device__ inline int32_t walker_lds_words(int32_t S, int32_t WW, int32_t FW, int32_t RS,
                                                    int32_t thr_words = kThrRow, int32_t acc_words = 4) {
  return gen_ring_words(S) + kMtN + FW + WW + 2 * RS + thr_words + acc_words;
}

// Two-field form: slot k's threshold row has one entry per pair (d_sp, d_t),
// d_sp in [-qds, qds] and d_t in [-qdt, qdt], at (d_sp + qds) * (2 qdt + 1) +
// d_t + qdt; rows longer than this are not supported.
constexpr int kMaxTwoFieldRow = 1024;

struct DevTables {
  const SysInfo *sys;
  const TmplSpin *tmpl;
  const uint32_t *thr;   // [slots][kThrRow]
  const double *beta;    // [slots]
  const Tile *tiles;
  const int32_t *walker_sys;  // [R] system of each walker
  const uint32_t *fifo;       // per template spin: (queue base << 8) | log2(queue depth)
  const uint16_t *lanes;      // per template: sweep lane position -> template spin
  const uint32_t *cells;      // per system, per phase: cells as (m << 16) | (y << 8) | x
  const int2 *cell_tiles;     // per 64-row tile of cell moves: its system, the walker of its first row
  const uint32_t *cellrec;    // cell records of the grid templates (see kCellRecWords)
  // two-field form: per-slot weights (a, c) and threshold rows of qrow words
  const uint32_t *qthr;       // [slots][qrow]
  const double *qa, *qc;      // [slots]
  int32_t two_field;          // 1: sweeps and swaps use the two-field form
  int32_t qrow, qwt, qoff;    // row words, 2 qdt + 1, qds * qwt + qdt
};

struct DevState {
  uint32_t *spins, *mt;
  int32_t *energy, *temp_of, *walker_at;
  uint32_t *swap_mt;
  uint64_t *flips, *swap_att, *swap_acc, *stats, *wsteps;
  int32_t *bond;  // running sum over tau edges of J_tau s s' (two-field form)
  uint64_t *swap_near;  // per pair (k, k+1), at slot k: swap decisions within 1e-12 of the threshold
};

// Raise the dynamic LDS limit of `kern` to `bytes`, once per device: bit d of
// `done` records device d (the attribute is set with that device current).
// Setting it is idempotent, so two threads racing here both just set it.
template <typename Kern>
inline hipError_t allow_lds(Kern kern, int bytes, std::atomic<uint64_t> &done) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const uint64_t bit = 1ull << (dev & 63);
  if (done.load(std::memory_order_acquire) & bit) return hipSuccess;
  e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) done.fetch_or(bit, std::memory_order_acq_rel);
  return e;
}

// Kernel launchers (each returns the hipError_t of the launch).
// Expand the seed stored in word 0 of every walker / swap stream window into
// the 624 init_genrand words.
hipError_t launch_seed(const DevState &s, int32_t R, int32_t n_sys, hipStream_t st);
hipError_t launch_sweep(const DevTables &t, const DevState &s, const Bucket &b, int32_t n_sweeps,
                        int32_t init_mode, hipStream_t st, LadderArgs la = LadderArgs{0, 0, 0, 0});
hipError_t launch_swap(const DevTables &t, const DevState &s, int32_t n_sys, int32_t parity,
                       int32_t *e_row, hipStream_t st);
hipError_t launch_record(const DevTables &t, const DevState &s, int32_t n_sys, int32_t *e_row,
                         hipStream_t st);
hipError_t launch_observables(const DevTables &t, const DevState &s, int32_t R, int32_t *obs,
                              int32_t set_energy, hipStream_t st);
hipError_t launch_cell_propose(const DevTables &t, const DevState &s, int32_t n_sys, int64_t rows_total,
                               int32_t phase, const float *w, const uint16_t *wb, uint64_t key, int64_t pass_index,
                               uint64_t *moves, hipStream_t st);
hipError_t launch_cell_heatbath(const DevTables &t, const DevState &s, int64_t rows_total, int32_t phase,
                                uint64_t key, int64_t pass_index, uint64_t *moves, hipStream_t st);
hipError_t launch_collect_cells(const DevTables &t, const DevState &s, int32_t n_sys, int64_t stride,
                                int64_t offset, int64_t total_cells, int32_t n, float *x, uint8_t *y,
                                hipStream_t st);
hipError_t launch_reduce_stats(const DevState &s, int32_t R, int32_t slots, hipStream_t st);
hipError_t launch_labels(const DevTables &t, const DevState &s, int32_t R, int32_t n_sys,
                         hipStream_t st);
// Layer-pair order: expand the seeds in row 0 of every generator lane
// (pair_mt is [kMtN][n_lanes]), and `n_sweeps` sweeps (init_mode: draw the
// initial spins) over every system, one workgroup per system, one launch per
// slice class present (bit 0: open slices, bit 1: a ring).
hipError_t launch_pair_seed(uint32_t *pair_mt, int64_t n_lanes, hipStream_t st);
hipError_t launch_pairs(const DevTables &t, const DevState &s, uint32_t *pair_mt, int64_t n_lanes, int32_t n_sys,
                        int32_t threads, size_t lds, uint32_t classes, int32_t n_sweeps, int32_t init_mode,
                        LadderArgs la, hipStream_t st);
// LDS words of one walker in the layer-pair kernel: M rows of RS spin words,
// threshold row, reduction words; odd, so the walkers of a wavefront use
// different banks.
__host__ __device__ inline int32_t pair_walker_words(int32_t WW) {
  const int32_t w = WW + kPairThrRow + 4;
  return w | 1;
}

}  // namespace ising
