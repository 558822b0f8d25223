// Cell moves: boundary fields of the 8-spin cells, training rows from the
// chain, the learned proposal with its Metropolis-Hastings test, and the exact
// heat-bath draw of a cell.
//
// A phase is one colour class of cells: cells of one colour share no edge, so
// all of them (in every walker) are updated at once; the phases run in order.
// Uniforms come from Philox4x32-10 (Salmon et al., SC'11): key (key mod 2^32,
// key div 2^32), counters (cell, walker, pass, j) for blocks j = 0, 1, 2; the
// words of blocks 0 and 1 are the 8 proposal uniforms, word 0 of block 2 the
// acceptance uniform.
#include "internal.h"
#include "mlp.h"

namespace ising {

// ---- Philox4x32-10 -----------------------------------------------------------
__device__ __forceinline__ void philox4x32(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c[0], p1 = (uint64_t)M1 * c[2];
    // three-input xor (bit-operation table 0x96) in one instruction
    const uint32_t x0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c[1], k0, 0x96);
    const uint32_t x2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c[3], k1, 0x96);
    c[0] = x0;
    c[1] = (uint32_t)p1;
    c[2] = x2;
    c[3] = (uint32_t)p0;
  }
}

// Last system whose first cell (walker-major numbering) is <= v.
__device__ __forceinline__ int find_system(const SysInfo *sys, int n_sys, int64_t v) {
  int lo = 0, hi = n_sys;  // invariant: answer in [lo, hi)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (sys[mid].cell0 <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Boundary fields b_k = h_k + sum_{j outside the cell} J_kj s_j of cell c of slice m.
// In-slice edges between cells join grid neighbours only (checked when the
// graph is loaded), so every outside neighbour in the slice lies in cell c - L,
// c + L, c - 1 or c + 1.  Their four bytes are packed into one word, and the
// cell record gives, for every outside neighbour, its coupling and its bit in
// that word; the tau neighbours are spin k of the cell in the slices before
// and after.
__device__ __forceinline__ void boundary_fields(const DevTables &T, const SysInfo &sy, const uint32_t *sp, int m,
                                                int c, int b[8], int32_t jpack[4] = nullptr) {
  const int M = sy.M, L = sy.grid_L;
  const int mp = m == 0 ? M - 1 : m - 1, mn = m == M - 1 ? 0 : m + 1;
  const bool has_p = M > 1 && (m > 0 || sy.ring), has_n = M > 1 && (m < M - 1 || sy.ring);
  const int y = c / L, x = c - (c / L) * L;
  const uint32_t *row = sp + m * sy.RS;
  const int cu = y > 0 ? c - L : c, cd = y < L - 1 ? c + L : c;
  const int cl = x > 0 ? c - 1 : c, cr = x < L - 1 ? c + 1 : c;
  auto cell_byte = [](uint32_t w, int cc) { return (w >> ((cc & 3) * 8)) & 0xffu; };
  const uint32_t nbytes = cell_byte(row[cu >> 2], cu) | (cell_byte(row[cd >> 2], cd) << 8) |
                          (cell_byte(row[cl >> 2], cl) << 16) | (cell_byte(row[cr >> 2], cr) << 24);
  const uint32_t bp = has_p ? cell_byte(sp[mp * sy.RS + (c >> 2)], c) : 0u;
  const uint32_t bn = has_n ? cell_byte(sp[mn * sy.RS + (c >> 2)], c) : 0u;
  const uint4 *rec = (const uint4 *)(T.cellrec + (size_t)(sy.cb0 + c) * kCellRecWords);
  const uint4 r0 = rec[0], r1 = rec[1], r2 = rec[2], r3 = rec[3], hq = rec[4], jq = rec[5];
  const uint32_t ent[16] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w,
                            r2.x, r2.y, r2.z, r2.w, r3.x, r3.y, r3.z, r3.w};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int f = (int)(int8_t)((((k < 4) ? hq.x : hq.y) >> (8 * (k & 3))) & 0xffu);
    const int jtau = (int)(int8_t)((((k < 4) ? hq.z : hq.w) >> (8 * (k & 3))) & 0xffu);
#pragma unroll
    for (int e = 0; e < 4; ++e) {  // an unused entry has J = 0
      const uint32_t v = ent[2 * k + (e >> 1)] >> (16 * (e & 1));
      const int J = (int)(int8_t)(v & 0xffu);
      const int bit = (int)((nbytes >> ((v >> 8) & 31u)) & 1u);
      f += J * (2 * bit - 1);
    }
    if (has_p) f += jtau * (2 * (int)((bp >> k) & 1u) - 1);
    if (has_n) f += jtau * (2 * (int)((bn >> k) & 1u) - 1);
    b[k] = f;
  }
  if (jpack) {
    jpack[0] = (int32_t)jq.x;
    jpack[1] = (int32_t)jq.y;
    jpack[2] = (int32_t)jq.z;
    jpack[3] = (int32_t)jq.w;
  }
}

__device__ __forceinline__ void write_features(float *x, const int b[8], float beta) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = 0.f;
    x[8 + k] = (float)b[k] * 0.125f;
  }
  x[16] = beta;
}

// E_c(s) = -sum_k b_k s_k - sum over in-cell edges J s s (bit k of `byte` = spin k is +1).
__device__ __forceinline__ int cell_energy(uint32_t byte, const int b[8], const int jin[16]) {
  int e = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) e -= b[k] * (((byte >> k) & 1u) ? 1 : -1);
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      e -= jin[k * 4 + i] * (((byte >> k) & 1u) ? 1 : -1) * (((byte >> (4 + i)) & 1u) ? 1 : -1);
  return e;
}

// E_c(s') - E_c(s) with packed byte products, for cell bytes s' = nb and s = cur
// (bit k = spin k is +1).  With s = 2 bit - 1, sum_k b_k s_k = 2 sum_k b_k bit_k
// - sum_k b_k, whose constant cancels in the difference, and for a left spin k,
// T_k = sum_r J_kr s_r = sum_r 2J_kr bit_r - jsum_k; each sum is one 4-way byte
// dot product.  blo / bhi hold b_0..b_3 / b_4..b_7 as signed bytes (|b| <= 63),
// jpack[k] the 2J of left spin k to right spins 0..3, njs[k] = -jsum_k.
__device__ __forceinline__ uint32_t spread4(uint32_t nib) { return __umul24(nib, 0x00204081u) & 0x01010101u; }

__device__ __forceinline__ int cell_delta_e(uint32_t nb, uint32_t cur, uint32_t blo, uint32_t bhi,
                                            const int32_t jpack[4], const int njs[4]) {
  const uint32_t rn = spread4(nb >> 4), rc = spread4(cur >> 4);
  const int bn = __builtin_amdgcn_sdot4((int)spread4(nb & 15u), (int)blo,
                                        __builtin_amdgcn_sdot4((int)rn, (int)bhi, 0, false), false);
  const int bc = __builtin_amdgcn_sdot4((int)spread4(cur & 15u), (int)blo,
                                        __builtin_amdgcn_sdot4((int)rc, (int)bhi, 0, false), false);
  int js = 0;  // sum_k s'_k T'_k - sum_k s_k T_k
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int tn = __builtin_amdgcn_sdot4((int)rn, jpack[k], njs[k], false);
    const int tc = __builtin_amdgcn_sdot4((int)rc, jpack[k], njs[k], false);
    js += (((nb >> k) & 1u) ? tn : -tn) - (((cur >> k) & 1u) ? tc : -tc);
  }
  return -2 * (bn - bc) - js;
}

// ---- rows of a colour class ---------------------------------------------------
// Row = (walker, cell of the class).  A 64-row tile lies in one system (rows
// of a system start at a multiple of 64); the fields of that system are read
// once per tile into wavefront-uniform registers.
struct CellRow {
  bool valid;
  int r, ci;           // global walker, cell index (m*L + y)*L + x
  int b[8];            // boundary fields (an invalid lane reads a clamped row; its values go unused)
  int32_t jpack[4];    // 2J of in-cell edges: spin k < 4 to spin 4 + i in byte i
  int njs[4];          // minus the sum over i of J between spin k < 4 and spin 4 + i
  float beta;
  int boff;            // byte offset of the cell's byte from the tile system's first spin word
  uint32_t cur;        // its current value (bit k = spin k is +1)
};

struct TileSys {
  int M, L, LL, RS, WW, ring, K, walker0, slot0, cb0, rows, cl0, p0, count, fast;
  int w0, j0;  // walker and cell-list position of the tile's first row
  long long spin_word0;
};

// A buffer resource over memory from a wavefront-uniform base: loads through
// it take a 32-bit byte offset per lane, so a lane's address needs no 64-bit
// arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_at(const void *p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ uint32_t load_b32(__amdgpu_buffer_rsrc_t r, int byte_off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0);
}
__device__ __forceinline__ uint4 load_b128(__amdgpu_buffer_rsrc_t r, int byte_off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0);
  return uint4{v[0], v[1], v[2], v[3]};
}

// Tables the kernels only read, through the scalar cache: with a uniform
// address the loads are scalar and land in scalar registers.
template <typename V>
__device__ __forceinline__ V load_uniform(const V *p) {
  return *(const __attribute__((address_space(4))) V *)p;
}

__device__ __forceinline__ TileSys tile_system(const DevTables &T, int64_t tile, int phase) {
  const long long td = load_uniform((const long long *)(T.cell_tiles + tile));  // {system, w0}
  const int sidx = (int)(uint32_t)td, w0 = (int)(td >> 32);
  const SysInfo *sy = T.sys + sidx;
  TileSys u;
  u.M = load_uniform(&sy->M);
  u.L = load_uniform(&sy->grid_L);
  u.LL = u.L * u.L;
  u.RS = load_uniform(&sy->RS);
  u.WW = load_uniform(&sy->WW);
  u.ring = load_uniform(&sy->ring);
  u.K = load_uniform(&sy->K);
  u.walker0 = load_uniform(&sy->walker0);
  u.slot0 = load_uniform(&sy->slot0);
  u.cb0 = load_uniform(&sy->cb0);
  u.rows = load_uniform(&sy->rows);
  u.cl0 = load_uniform(&sy->cl0);
  u.fast = load_uniform(&sy->cell_fast);
  const int np = load_uniform(&sy->n_phases);
  u.p0 = phase < np ? load_uniform(&sy->pc[phase]) : 0;
  u.count = phase < np ? load_uniform(&sy->pc[phase + 1]) - u.p0 : 0;
  u.spin_word0 = load_uniform(&sy->spin_word0);
  u.w0 = w0;
  u.j0 = (int)(tile * 64 - load_uniform(&sy->row0)) - w0 * u.rows;
  return u;
}

// The lane's row: its walker and cell, the cell's boundary fields b_k = h_k +
// sum_{j outside the cell} J_kj s_j, in-cell couplings, byte and beta.  Every
// load is issued before any is used: the cell list entry and the walker's
// slot, then the seven spin words around the cell (the cells above, below,
// left and right in its slice, the cell itself, and the cell in the slices
// before and after), its record and beta.  In-slice edges between cells join
// grid neighbours only (checked when the graph is loaded), so a neighbour's
// bit lies in one word that packs the four neighbour cells' bytes.  With
// cell_fast the neighbours of spin k are spin k of each neighbour cell: the
// four bits are (word >> k) & 0x01010101 and one byte dot product with the
// couplings by direction sums them; otherwise each of the record's entries
// names the neighbour's bit.
__device__ __forceinline__ void load_row(const DevTables &T, const DevState &St, const TileSys &u, int lane,
                                         CellRow &c) {
  // rows are walker-major, `rows` per walker: the tile's first row is (w0, j0)
  int wk = u.w0, j = u.j0 + lane;
  if (u.rows >= 64) {  // at most one walker boundary in the tile
    const bool next = j >= u.rows;
    wk += next ? 1 : 0;
    j -= next ? u.rows : 0;
  } else {
    const int q = j / u.rows;
    wk += q;
    j -= q * u.rows;
  }
  c.valid = wk < u.K && j < u.count;
  const int wkc = c.valid ? wk : 0, jc = c.valid ? j : 0;
  c.r = c.valid ? u.walker0 + wk : -1;
  const uint32_t pc = load_b32(buffer_at(T.cells + u.cl0 + u.p0), 4 * jc);
  const int tof = (int)load_b32(buffer_at(St.temp_of + u.walker0), 4 * wkc);
  const int m = (int)(pc >> 16), y = (int)((pc >> 8) & 0xffu), x = (int)(pc & 0xffu);
  // (the products below are of small counts: 24-bit multiplies, full rate)
  const int cc = __mul24(y, u.L) + x;
  c.ci = __mul24(m, u.LL) + cc;
  // spin words from the system's first one: walker wkc, row m, word (cell >> 2)
  const __amdgpu_buffer_rsrc_t spins = buffer_at(St.spins + u.spin_word0);
  const int wofs = __mul24(wkc, u.WW), row = 4 * (wofs + __mul24(m, u.RS));
  const int mp = m == 0 ? u.M - 1 : m - 1, mn = m == u.M - 1 ? 0 : m + 1;
  const bool has_p = u.M > 1 && (m > 0 || u.ring), has_n = u.M > 1 && (m < u.M - 1 || u.ring);
  const int cu = y > 0 ? cc - u.L : cc, cd = y < u.L - 1 ? cc + u.L : cc;
  const int cl = x > 0 ? cc - 1 : cc, cr = x < u.L - 1 ? cc + 1 : cc;
  const uint32_t wu = load_b32(spins, row + 4 * (cu >> 2)), wdn = load_b32(spins, row + 4 * (cd >> 2)),
                 wl = load_b32(spins, row + 4 * (cl >> 2)), wr = load_b32(spins, row + 4 * (cr >> 2)),
                 wo = load_b32(spins, row + 4 * (cc >> 2));
  const uint32_t wp = load_b32(spins, 4 * (wofs + __mul24(mp, u.RS) + (cc >> 2))),
                 wn = load_b32(spins, 4 * (wofs + __mul24(mn, u.RS) + (cc >> 2)));
  // the cell's record: uint4 i at byte 16 i
  const __amdgpu_buffer_rsrc_t recs = buffer_at(T.cellrec + (size_t)u.cb0 * kCellRecWords);
  const int ro = __mul24(cc, 4 * kCellRecWords);
  const uint4 hq = load_b128(recs, ro + 64), jq = load_b128(recs, ro + 80);
  auto cell_byte = [](uint32_t w, int q) { return (w >> ((q & 3) * 8)) & 0xffu; };
  const uint32_t nbytes = cell_byte(wu, cu) | (cell_byte(wdn, cd) << 8) | (cell_byte(wl, cl) << 16) |
                          (cell_byte(wr, cr) << 24);
  const uint32_t bp = has_p ? cell_byte(wp, cc) : 0u, bn = has_n ? cell_byte(wn, cc) : 0u;
  const uint4 hx = load_b128(recs, ro + 128);
  if (u.fast) {
    // f_k = h''_k + sum_dir 2J bit + jtau_k U_k, with h''_k = h_k - sum_dir J - 2 jtau_k
    // from the record and U_k = 2 (bit k of the slice before, if any) + 2 (bit k
    // of the slice after, if any) + the number of missing tau neighbours, built
    // for all eight spins as bytes (0..4, no carries)
    const uint4 d0 = load_b128(recs, ro + 96), d1 = load_b128(recs, ro + 112);
    const uint32_t dir[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
    const uint32_t pm = has_p ? bp : 0u, nm = has_n ? bn : 0u;
    const uint32_t miss = (has_p ? 0u : 0x01010101u) + (has_n ? 0u : 0x01010101u);
    const uint32_t U[2] = {2u * (spread4(pm & 15u) + spread4(nm & 15u)) + miss,
                           2u * (spread4(pm >> 4) + spread4(nm >> 4)) + miss};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int h2 = (int)(int8_t)((((k < 4) ? hx.x : hx.y) >> (8 * (k & 3))) & 0xffu);
      const int jtau = (int)(int8_t)((((k < 4) ? hq.z : hq.w) >> (8 * (k & 3))) & 0xffu);
      const int uk = (int)((U[k >> 2] >> (8 * (k & 3))) & 0xffu);
      c.b[k] = __builtin_amdgcn_sdot4((int)((nbytes >> k) & 0x01010101u), (int)dir[k], h2, false) + jtau * uk;
    }
  } else {
    const uint4 r0 = load_b128(recs, ro), r1 = load_b128(recs, ro + 16), r2 = load_b128(recs, ro + 32),
                r3 = load_b128(recs, ro + 48);
    const uint32_t ent[16] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w,
                              r2.x, r2.y, r2.z, r2.w, r3.x, r3.y, r3.z, r3.w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int f = (int)(int8_t)((((k < 4) ? hq.x : hq.y) >> (8 * (k & 3))) & 0xffu);
      const int jtau = (int)(int8_t)((((k < 4) ? hq.z : hq.w) >> (8 * (k & 3))) & 0xffu);
#pragma unroll
      for (int e = 0; e < 4; ++e) {  // an unused entry has J = 0
        const uint32_t v = ent[2 * k + (e >> 1)] >> (16 * (e & 1));
        const int J = (int)(int8_t)(v & 0xffu);
        const int bit = (int)((nbytes >> ((v >> 8) & 31u)) & 1u);
        f += J * (2 * bit - 1);
      }
      if (has_p) f += jtau * (2 * (int)((bp >> k) & 1u) - 1);
      if (has_n) f += jtau * (2 * (int)((bn >> k) & 1u) - 1);
      c.b[k] = c.valid ? f : 0;
    }
  }
  c.jpack[0] = (int32_t)jq.x;
  c.jpack[1] = (int32_t)jq.y;
  c.jpack[2] = (int32_t)jq.z;
  c.jpack[3] = (int32_t)jq.w;
  c.njs[0] = (int)(int16_t)(hx.z & 0xffffu);
  c.njs[1] = (int)(int32_t)hx.z >> 16;
  c.njs[2] = (int)(int16_t)(hx.w & 0xffffu);
  c.njs[3] = (int)(int32_t)hx.w >> 16;
  c.boff = row + cc;  // word cc >> 2 of the row, byte cc & 3
  c.cur = cell_byte(wo, cc);
  const double beta = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(buffer_at(T.beta + u.slot0), 8 * tof, 0, 0));
  c.beta = c.valid ? (float)beta : 0.f;
}

// This wavefront's tiles: a contiguous run (the rows of one walker, then the
// next), so a walker's spin words and its system's records stay in cache.
struct TileRange {
  int64_t begin, end;
};
__device__ __forceinline__ TileRange wave_tiles(int64_t tiles, int waves_per_group) {
  const int64_t nwaves = (int64_t)gridDim.x * waves_per_group;
  const int64_t per = (tiles + nwaves - 1) / nwaves;
  // the wavefront's index, read from lane 0: the compiler then knows the range is
  // uniform, keeps the tile loop in scalar registers and loads the tile's tables
  // through the scalar cache
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t w = (int64_t)blockIdx.x * waves_per_group + wave;
  const int64_t b = w * per;
  return TileRange{b < tiles ? b : tiles, b + per < tiles ? b + per : tiles};
}

// Per-walker sums of a wavefront's rows: energy change, rows, rows counted in
// `hit`; one atomic each when the lanes share a walker.
__device__ __forceinline__ void add_cell_moves(const DevState &St, uint64_t *moves, int r, bool valid, bool hit,
                                               int dE, int lane) {
  const int r0 = __shfl(r, 0);
  const bool uniform = __all(r == r0);
  if (uniform) {
    if (r0 >= 0) {
      int tot = dE;
      for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
      const unsigned long long na = __popcll(__ballot(valid && hit));
      const unsigned long long nv = __popcll(__ballot(valid));
      if (lane == 0) {
        if (tot) atomicAdd(&St.energy[r0], tot);
        if (moves) {
          atomicAdd((unsigned long long *)&moves[2 * (size_t)r0], nv);
          atomicAdd((unsigned long long *)&moves[2 * (size_t)r0 + 1], na);
        }
      }
    }
  } else if (valid) {
    if (dE) atomicAdd(&St.energy[r], dE);
    if (moves) {
      atomicAdd((unsigned long long *)&moves[2 * (size_t)r], 1ull);
      if (hit) atomicAdd((unsigned long long *)&moves[2 * (size_t)r + 1], 1ull);
    }
  }
}

// ---- one colour class of cell moves in one launch -----------------------------
// Each wavefront takes tiles of 64 rows (row = walker x cell of the class, one
// lane per row): the lane computes its cell's boundary fields and writes the
// BF16 network input to LDS; the three layers run on BF16 matrix cores with the
// rows as the N side (16-row tiles), so that a layer's results stay in the
// lanes that feed them to the next layer; the logits go back through LDS to the
// row's lane, which draws the proposal and takes the Metropolis-Hastings
// decision.
//
// Result tiles: lane l holds units 4(l/16) + j (j < 4) of row l % 16.  The
// next layer's B operand wants, in lane l, 8 consecutive positions of the
// contraction axis for row l % 16; the contraction order is free, so position
// 32kk + 8g + p (g = l/16) is taken to be unit 32kk + 4g + p for p < 4 and
// 32kk + 16 + 4g + (p - 4) for p >= 4 -- exactly what the lane holds from
// result tiles 2kk and 2kk + 1 -- and the weight columns are stored in that
// order.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int unit_at(int c) {
  const int kk = c >> 5, g = (c >> 3) & 3, p = c & 7;
  return (kk << 5) + (p < 4 ? 4 * g + p : 16 + 4 * g + (p - 4));
}

// Row strides are padded by 8 BF16 (16 bytes): the 16 rows that one matrix
// operand read touches then fall on distinct LDS banks.
constexpr int kS2 = 136;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

typedef short i16x2 __attribute__((ext_vector_type(2)));

// relu of two FP32 values, as packed BF16 (round to nearest even).  The
// rounding keeps the sign, so relu is applied after it: read as 16-bit
// integers, BF16 values below zero (and -0) are negative, and a packed
// integer max with 0 clears exactly those.
__device__ __forceinline__ uint32_t relu_bf2(float a, float b) {
  const i16x2 v = __builtin_bit_cast(i16x2, __builtin_convertvector((f32x2{a, b}), bf16x2));
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, (i16x2{0, 0})));
}

__device__ __forceinline__ uint32_t pack_bf2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{a, b}), bf16x2));
}

__device__ __forceinline__ f32x4 mfma16(u32x4 a, u32x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                  0, 0);
}

// Occupancy: eight wavefronts per workgroup share one LDS copy of the weights
// (69 KiB with their inputs), two workgroups per CU, four wavefronts per SIMD
// (at most 128 VGPRs).  To fit, layer 1 takes only the 9 non-zero inputs (b/8
// and beta; the 8 spin slots are zero) as a 16-wide contraction (16x16x16
// MFMA; the zero inputs contributed nothing: a pass of the 32-wide form gave
// the same spins and energies bit for bit), and the network runs on the 64
// rows in two halves of 32, so only one half's layer-1 activations (32 VGPRs)
// are live at a time; each half reads the layer-2 weights again.
constexpr int kProposeWaves = 8;
constexpr int kX2 = 24;  // input row stride (bf16): 16 positions + 8 padding
struct alignas(16) ProposeLds {
  uint16_t W1[128 * kX2];  // [unit][position]: b0..b7, beta, zeros
  uint16_t W2[128 * kS2];  // [unit][position], positions in unit_at order
  uint16_t W3[16 * kS2];   // [output (8 + 8 zero rows)][position]
  float b1[128], b2[128], b3[16];
  uint16_t X[kProposeWaves][64 * kX2];  // per wavefront: inputs of its 64 rows, then their logits
};
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 mfma16k16(u32x2 a, u32x2 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a), __builtin_bit_cast(s16x4, b), c, 0,
                                                   0, 0);
}

__global__ void __launch_bounds__(64 * kProposeWaves) __attribute__((amdgpu_waves_per_eu(4)))
    cell_propose_kernel(DevTables T, DevState St, int32_t n_sys, int64_t rows_total, int32_t phase, const float *w,
                         const uint16_t *wb, uint64_t key, int64_t pass_index, uint64_t *moves) {
  __shared__ ProposeLds s;
  // W1: inputs 8..16 of the packed rows (b0..b7, beta) to positions 0..8
  for (int i = threadIdx.x; i < 128 * kX2; i += blockDim.x) {
    const int u = i / kX2, p = i - u * kX2;
    s.W1[i] = p < 9 ? wb[kPW1 + u * 32 + 8 + p] : (uint16_t)0;
  }
  for (int i = threadIdx.x; i < 144 * 16; i += blockDim.x) {
    const int row = i >> 4, kk = (i >> 2) & 3, gg = i & 3;
    const uint16_t *src = row < 128 ? wb + kPW2 + row * 128 : wb + kPW3 + (row - 128) * 128;
    uint16_t *dst = row < 128 ? s.W2 + row * kS2 : s.W3 + (row - 128) * kS2;
    const uint2 a = *(const uint2 *)(src + kk * 32 + 4 * gg), b = *(const uint2 *)(src + kk * 32 + 16 + 4 * gg);
    *(uint4 *)(dst + kk * 32 + gg * 8) = uint4{a.x, a.y, b.x, b.y};
  }
  for (int i = threadIdx.x; i < 128; i += blockDim.x) {
    s.b1[i] = w[kOB1 + i];
    s.b2[i] = w[kOB2 + i];
  }
  for (int i = threadIdx.x; i < 16; i += blockDim.x) s.b3[i] = i < kOut ? w[kOB3 + i] : 0.f;
  __syncthreads();

  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, n16 = l & 15, g = l >> 4;
  uint16_t *X = s.X[wv];
  float *Lg = (float *)X;
  const TileRange tr = wave_tiles(rows_total / 64, kProposeWaves);
  for (int64_t tile = tr.begin; tile < tr.end; ++tile) {
    CellRow cr;
    const TileSys ts = tile_system(T, tile, phase);
    load_row(T, St, ts, l, cr);
    const bool valid = cr.valid;
    const int *b = cr.b;
    const float beta = cr.beta;
    {
      u32x4 *xr = (u32x4 *)(X + l * kX2);
      xr[0] = u32x4{pack_bf2(b[0] * 0.125f, b[1] * 0.125f), pack_bf2(b[2] * 0.125f, b[3] * 0.125f),
                    pack_bf2(b[4] * 0.125f, b[5] * 0.125f), pack_bf2(b[6] * 0.125f, b[7] * 0.125f)};
      xr[1] = u32x4{(uint32_t)f2bf(beta), 0u, 0u, 0u};
    }
    wave_fence();
    // A wavefront in the network raises its priority, so its matrix-core work
    // is issued first and the other wavefronts' vector work fills around it
    // (3-4% faster than without; forcing two wavefront groups into opposite
    // phases with barriers was slower).
    __builtin_amdgcn_s_setprio(1);
    const f32x4 bias3 = *(const f32x4 *)(s.b3 + 4 * (g & 3));
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      u32x2 xb[2];
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) xb[tt] = *(const u32x2 *)(X + ((2 * half + tt) * 16 + n16) * kX2 + g * 4);
      u32x4 h1[4][2];
#pragma unroll
      for (int ft = 0; ft < 8; ++ft) {
        const u32x2 a = *(const u32x2 *)(s.W1 + (ft * 16 + n16) * kX2 + g * 4);
        const f32x4 bias = *(const f32x4 *)(s.b1 + ft * 16 + 4 * g);
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
          const f32x4 acc = mfma16k16(a, xb[tt], bias);
          h1[ft >> 1][tt][(ft & 1) * 2] = relu_bf2(acc[0], acc[1]);
          h1[ft >> 1][tt][(ft & 1) * 2 + 1] = relu_bf2(acc[2], acc[3]);
        }
      }
      f32x4 acc3[2] = {bias3, bias3};
#pragma unroll
      for (int kk3 = 0; kk3 < 4; ++kk3) {
        u32x4 h2[2];
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
          const int ft = 2 * kk3 + hf;
          u32x4 wa[4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) wa[kk] = *(const u32x4 *)(s.W2 + (ft * 16 + n16) * kS2 + kk * 32 + g * 8);
          const f32x4 bias = *(const f32x4 *)(s.b2 + ft * 16 + 4 * g);
          f32x4 acc[2] = {bias, bias};
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) acc[tt] = mfma16(wa[kk], h1[kk][tt], acc[tt]);
#pragma unroll
          for (int tt = 0; tt < 2; ++tt) {
            h2[tt][hf * 2] = relu_bf2(acc[tt][0], acc[tt][1]);
            h2[tt][hf * 2 + 1] = relu_bf2(acc[tt][2], acc[tt][3]);
          }
        }
        const u32x4 a3 = *(const u32x4 *)(s.W3 + n16 * kS2 + kk3 * 32 + g * 8);
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) acc3[tt] = mfma16(a3, h2[tt], acc3[tt]);
      }
      // this half's logits: rows 32 half .. 32 half + 31 take bytes 1 KB half of the region,
      // which only holds inputs of rows already read (rows below 22 (half 0) or 43 (half 1))
      wave_fence();
      if (g < 2) {
#pragma unroll
        for (int tt = 0; tt < 2; ++tt)
#pragma unroll
          for (int j = 0; j < 4; ++j) Lg[((2 * half + tt) * 16 + n16) * 8 + 4 * g + j] = acc3[tt][j];
      }
    }
    __builtin_amdgcn_s_setprio(0);
    wave_fence();

    int dE = 0;
    bool accept = false;
    if (valid) {
      float lg[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) lg[k] = Lg[l * 8 + k];
      const uint32_t cur = cr.cur;
      const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
      uint32_t wd[12];
#pragma unroll
      for (int blk = 0; blk < 3; ++blk) {
        uint32_t c4[4] = {(uint32_t)cr.ci, (uint32_t)cr.r, (uint32_t)pass_index, (uint32_t)blk};
        philox4x32(c4, k0, k1);
#pragma unroll
        for (int q = 0; q < 4; ++q) wd[4 * blk + q] = c4[q];
      }
      uint32_t nb = 0;
      float lratio = 0.f;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        // u (1 + e^-l) < 1 with u = word 2^-32, scaled by 2^32 (exact in FP32)
        const bool up = (float)wd[k] * (1.f + __expf(-lg[k])) < 0x1p32f;
        nb |= (up ? 1u : 0u) << k;
        const bool was_up = (cur >> k) & 1u;
        if (up != was_up) lratio += was_up ? lg[k] : -lg[k];
      }
      {
        uint32_t blo = 0, bhi = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          blo |= (uint32_t)(b[k] & 0xff) << (8 * k);
          bhi |= (uint32_t)(b[4 + k] & 0xff) << (8 * k);
        }
        dE = cell_delta_e(nb, cur, blo, bhi, cr.jpack, cr.njs);
      }
      const float la = -beta * (float)dE + lratio;
      const float ua = (float)wd[8] * 0x1p-32f;
      accept = la >= 0.f || ua < __expf(la);
      if (accept && nb != cur)
        __builtin_amdgcn_raw_buffer_store_b8((uint8_t)nb, buffer_at(St.spins + ts.spin_word0), cr.boff, 0, 0);
      if (!accept) dE = 0;
    }
    wave_fence();
    add_cell_moves(St, moves, cr.r, valid, accept, dE, l);
  }
}

hipError_t launch_cell_propose(const DevTables &t, const DevState &s, int32_t n_sys, int64_t rows_total,
                               int32_t phase, const float *w, const uint16_t *wb, uint64_t key, int64_t pass_index,
                               uint64_t *moves, hipStream_t st) {
  if (rows_total <= 0) return hipSuccess;
  const int64_t tiles = rows_total / 64;
  const int blocks = (int)std::min<int64_t>((tiles + kProposeWaves - 1) / kProposeWaves, 512);
  hipLaunchKernelGGL(cell_propose_kernel, dim3(blocks), dim3(64 * kProposeWaves), 0, st, t, s, n_sys, rows_total,
                     phase, w, wb, key, pass_index, moves);
  return hipGetLastError();
}

// ---- exact heat-bath cell moves (the non-learned control) ----------------------
// A cell is redrawn from its conditional Boltzmann law given the boundary.  The
// cell is bipartite, so: the left half (spins 0..3) from its marginal over 16
// states, log weight beta sum_k b_k s_k + sum_r log(2 cosh(beta h_r)),
// h_r = b_r + sum_k J_kr s_k; then each right spin r with P(+1) =
// sigmoid(2 beta h_r).  Words of Philox4x32-10 blocks (cell, walker, pass, 0..1):
// word 0 picks the left state by its cumulative weight, words 1..4 the right
// spins.  FP32 with the hardware exp/log.
__global__ void __launch_bounds__(256) cell_heatbath_kernel(DevTables T, DevState St, int64_t rows_total,
                                                            int32_t phase, uint64_t key, int64_t pass_index,
                                                            uint64_t *moves) {
  const int l = threadIdx.x & 63;
  const TileRange tr = wave_tiles(rows_total / 64, 4);
  for (int64_t tile = tr.begin; tile < tr.end; ++tile) {
    CellRow cr;
    const TileSys ts = tile_system(T, tile, phase);
    load_row(T, St, ts, l, cr);
    int dE = 0;
    bool changed = false;
    if (cr.valid) {
      const int *b = cr.b;
      const float bt = cr.beta;
      int jin[16];  // J between left spin k and right spin 4 + i at [k*4 + i]
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i) jin[k * 4 + i] = ((int32_t)(int8_t)((cr.jpack[k] >> (8 * i)) & 0xff)) / 2;
      float lw[16];
      float mx = -3.0e38f;
#pragma unroll
      for (int li = 0; li < 16; ++li) {
        int sb = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) sb += ((li >> k) & 1) ? b[k] : -b[k];
        float a = bt * (float)sb;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int h = b[4 + r];
#pragma unroll
          for (int k = 0; k < 4; ++k) h += ((li >> k) & 1) ? jin[k * 4 + r] : -jin[k * 4 + r];
          const float x = bt * fabsf((float)h);
          a += x + __logf(1.f + __expf(-2.f * x));  // log(2 cosh x)
        }
        lw[li] = a;
        mx = fmaxf(mx, a);
      }
      const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
      uint32_t wd[8];
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) {
        uint32_t c4[4] = {(uint32_t)cr.ci, (uint32_t)cr.r, (uint32_t)pass_index, (uint32_t)blk};
        philox4x32(c4, k0, k1);
#pragma unroll
        for (int q = 0; q < 4; ++q) wd[4 * blk + q] = c4[q];
      }
      float cum[16];
      float tot = 0.f;
#pragma unroll
      for (int li = 0; li < 16; ++li) {
        tot += __expf(lw[li] - mx);
        cum[li] = tot;
      }
      const float target = (float)wd[0] * 0x1p-32f * tot;
      int left = 0;  // the first state whose cumulative weight exceeds the target
#pragma unroll
      for (int li = 0; li < 16; ++li) left += cum[li] <= target ? 1 : 0;
      left = left > 15 ? 15 : left;
      uint32_t nb = (uint32_t)left;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int h = b[4 + r];
#pragma unroll
        for (int k = 0; k < 4; ++k) h += ((left >> k) & 1) ? jin[k * 4 + r] : -jin[k * 4 + r];
        const float p = 1.f / (1.f + __expf(-2.f * bt * (float)h));
        nb |= ((float)wd[1 + r] * 0x1p-32f < p ? 1u : 0u) << (4 + r);
      }
      dE = cell_energy(nb, b, jin) - cell_energy(cr.cur, b, jin);
      changed = nb != cr.cur;
      if (changed)
        __builtin_amdgcn_raw_buffer_store_b8((uint8_t)nb, buffer_at(St.spins + ts.spin_word0), cr.boff, 0, 0);
    }
    add_cell_moves(St, moves, cr.r, cr.valid, changed, dE, l);
  }
}

hipError_t launch_cell_heatbath(const DevTables &t, const DevState &s, int64_t rows_total, int32_t phase,
                                uint64_t key, int64_t pass_index, uint64_t *moves, hipStream_t st) {
  if (rows_total <= 0) return hipSuccess;
  const int64_t tiles = rows_total / 64;
  const int blocks = (int)std::min<int64_t>((tiles + 3) / 4, 2048);
  hipLaunchKernelGGL(cell_heatbath_kernel, dim3(blocks), dim3(256), 0, st, t, s, rows_total, phase, key, pass_index,
                     moves);
  return hipGetLastError();
}

// ---- training rows from the current spins ------------------------------------
__global__ void collect_cells_kernel(DevTables T, DevState St, int32_t n_sys, int64_t stride, int64_t offset,
                                     int64_t total_cells, int32_t n, float *X, uint8_t *Y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t g = (offset + (int64_t)i * stride) % total_cells;
  const SysInfo sy = T.sys[find_system(T.sys, n_sys, g)];
  const int LL = sy.grid_L * sy.grid_L;
  const int64_t per_walker = (int64_t)sy.M * LL;
  const int64_t local = g - sy.cell0;
  const int w = (int)(local / per_walker), ci = (int)(local % per_walker);
  const int m = ci / LL, c = ci - m * LL;
  const uint32_t *sp = St.spins + sy.spin_word0 + (size_t)w * sy.WW;
  int b[8];
  boundary_fields(T, sy, sp, m, c, b);
  write_features(X + (int64_t)i * kIn, b, (float)T.beta[sy.slot0 + St.temp_of[sy.walker0 + w]]);
  Y[i] = (uint8_t)((sp[m * sy.RS + ((c * 8) >> 5)] >> ((c * 8) & 31)) & 0xffu);
}

hipError_t launch_collect_cells(const DevTables &t, const DevState &s, int32_t n_sys, int64_t stride,
                                int64_t offset, int64_t total_cells, int32_t n, float *x, uint8_t *y,
                                hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(collect_cells_kernel, dim3((n + 255) / 256), dim3(256), 0, st, t, s, n_sys, stride, offset,
                     total_cells, n, x, y);
  return hipGetLastError();
}

}  // namespace ising
