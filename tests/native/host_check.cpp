// Host-only checks of libising's planning code, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers.py (no GPU, no HIP
// runtime call): validation and packing of systems of every workload shape and
// of invalid ones, the cell records of grid templates, every launch shape of
// every bucket with its tiles and sweep limit, and the threshold, acceptance and
// two-field rows.  Prints one line per
// case and "host_check OK" at the end; any failed check exits non-zero.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <string>
#include <vector>

#include "host.h"

using namespace ising;

#define CHECK(c)                                                           \
  do {                                                                     \
    if (!(c)) {                                                            \
      fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #c, \
              ising_last_error());                                         \
      exit(1);                                                             \
    }                                                                      \
  } while (0)

struct Rng {  // xorshift64*: inputs only
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed * 2685821657736338717ull + 1) {}
  uint32_t next() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return (uint32_t)((s * 2685821657736338717ull) >> 32);
  }
  int8_t coupling() {
    static const int8_t v[6] = {-3, -2, -1, 1, 2, 3};
    return v[next() % 6];
  }
};

struct Sys {
  int32_t S = 0, M = 1, ring = 0;
  std::vector<int32_t> u, v;
  std::vector<int8_t> J, h, jt;
  std::vector<double> beta;
  ising_system_desc desc() const {
    return ising_system_desc{S, M, ring, (int32_t)u.size(), u.data(), v.data(), J.data(), h.data(),
                             jt.data(), (int32_t)beta.size(), beta.data()};
  }
};

static std::vector<double> ladder(int K, double lo, double hi) {
  std::vector<double> b(K);
  for (int k = 0; k < K; ++k) b[k] = K == 1 ? hi : lo * pow(hi / lo, (double)k / (K - 1));
  return b;
}

// L x L grid of K4,4 cells, M slices (the workload shape of the paper's QMC models).
static Sys chimera(int L, int M, int K, uint64_t seed, bool ring = true) {
  Sys s;
  Rng r(seed);
  s.S = 8 * L * L;
  s.M = M;
  s.ring = ring ? 1 : 0;
  auto cell = [&](int y, int x) { return (y * L + x) * 8; };
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x)
      for (int k = 0; k < 4; ++k)
        for (int k2 = 4; k2 < 8; ++k2) s.u.push_back(cell(y, x) + k), s.v.push_back(cell(y, x) + k2);
  for (int y = 0; y + 1 < L; ++y)
    for (int x = 0; x < L; ++x)
      for (int k = 0; k < 4; ++k) s.u.push_back(cell(y, x) + k), s.v.push_back(cell(y + 1, x) + k);
  for (int y = 0; y < L; ++y)
    for (int x = 0; x + 1 < L; ++x)
      for (int k = 4; k < 8; ++k) s.u.push_back(cell(y, x) + k), s.v.push_back(cell(y, x + 1) + k);
  for (int q = 0; q < s.S; ++q) s.h.push_back(r.coupling());
  for (size_t e = 0; e < s.u.size(); ++e) s.J.push_back(r.coupling());
  for (int q = 0; q < s.S; ++q) s.jt.push_back(r.coupling());
  s.beta = ladder(K, 0.1, 3.0);
  return s;
}

static Sys random_graph(int N, int nE, int K, uint64_t seed, int maxdeg = 8) {
  Sys s;
  Rng r(seed);
  s.S = N;
  std::vector<int> deg(N, 0);
  std::vector<std::vector<char>> seen(N, std::vector<char>(N, 0));
  for (int t = 0; t < 100000 && (int)s.u.size() < nE && N > 1; ++t) {
    int a = r.next() % N, b = r.next() % N;
    if (a == b || seen[a][b] || deg[a] >= maxdeg || deg[b] >= maxdeg) continue;
    seen[a][b] = seen[b][a] = 1;
    ++deg[a], ++deg[b];
    s.u.push_back(a), s.v.push_back(b), s.J.push_back(r.coupling());
  }
  for (int q = 0; q < N; ++q) s.h.push_back(r.coupling()), s.jt.push_back(0);
  s.beta = ladder(K, 0.1, 3.0);
  return s;
}

// Cell records of a grid template against sums taken straight from the system
// description: the constant part of each spin's boundary field, h - sum of J to
// its neighbours outside the cell - 2 J_tau (when the records carry couplings by
// direction), and minus the sum of J from each left spin to the right spins of
// its cell.
static void check_cell_records(const Sys &s, const SysHost &hs) {
  if (hs.grid_L == 0) return;
  std::vector<int> out(s.S, 0), in(s.S, 0);
  for (size_t e = 0; e < s.u.size(); ++e) {
    const int a = s.u[e], b = s.v[e];
    if ((a >> 3) == (b >> 3)) {
      in[(a & 4) ? b : a] += s.J[e];
    } else {
      out[a] += s.J[e];
      out[b] += s.J[e];
    }
  }
  for (int c = 0; c < s.S / 8; ++c) {
    const uint32_t *rec = hs.cellrec.data() + (size_t)c * kCellRecWords;
    for (int k = 0; k < 8; ++k) {
      const int q = 8 * c + k;
      const int hc = s.h[q] - out[q] - 2 * s.jt[q];
      if (hs.cell_fast) CHECK((int)(int8_t)(uint8_t)(rec[32 + (k >> 2)] >> (8 * (k & 3))) == hc);
      if (k < 4) CHECK((int)(int16_t)(uint16_t)(rec[34 + (k >> 1)] >> (16 * (k & 1))) == -in[q]);
    }
  }
}

// Plan a batch and try every launch shape of every bucket: tiles must cover
// each walker of the bucket's systems exactly once.
static void check_batch(const char *name, const std::vector<Sys> &systems) {
  std::vector<ising_system_desc> d;
  for (const Sys &s : systems) d.push_back(s.desc());
  size_t bytes = 0;
  CHECK(ising_graph_bytes(d.data(), (int32_t)d.size(), &bytes) == ISING_OK);
  std::vector<SysHost> hs;
  CHECK(build_all(d.data(), (int32_t)d.size(), hs) == ISING_OK);
  for (size_t i = 0; i < systems.size(); ++i) check_cell_records(systems[i], hs[i]);
  GraphPlan g;
  CHECK(plan(hs, g) == ISING_OK);
  const int64_t default_limit = sweep_limit(g);
  int shapes = 0;
  for (size_t bi = 0; bi < g.buckets.size(); ++bi) {
    int32_t Kmax = 1;
    for (int32_t s : g.bucket_sys[bi]) Kmax = std::max(Kmax, g.sys[s].K);
    const Bucket orig = g.buckets[bi];
    std::vector<int32_t> tpws = tpw_candidates(orig.S);
    for (int32_t t : {1, 2, 4, 2048, 63, 65, 100, 1025}) tpws.push_back(t);  // also invalid ones
    for (int32_t tpw : tpws)
      for (int32_t G = 1; G <= 64; G <<= 1) {
        Bucket b = orig;
        if (shape_bucket(b, tpw, G, Kmax, true) != ISING_OK) {
          CHECK(tpw > 1024 || (tpw <= 64 && (tpw & (tpw - 1))) || b.S > tpw * 8 || G * tpw > 1024 ||
                (tpw > 64 && tpw % 64 && b.S > tpw * 2) ||
                (size_t)G * b.walker_words * 4 > 160 * 1024);
          continue;
        }
        CHECK(b.cpt >= 1 && b.cpt <= 8 && (int64_t)b.tpw * b.cpt >= b.S);
        CHECK(b.tpw <= 64 || b.tpw % 64 == 0 || b.cpt <= 2);
        CHECK(b.threads % 64 == 0 && b.threads <= 1024 && b.lds <= 160 * 1024);
        g.buckets[bi] = b;
        retile(g);
        std::vector<int> seen(g.R, 0);
        for (const Bucket &bk : g.buckets)
          for (int32_t t = bk.tile0; t < bk.tile0 + bk.ntiles; ++t) {
            const Tile &tl = g.tiles[t];
            CHECK(tl.nw >= 1 && tl.nw <= bk.G && tl.w0 + tl.nw <= g.sys[tl.sys].K);
            for (int32_t w = 0; w < tl.nw; ++w) ++seen[g.sys[tl.sys].walker0 + tl.w0 + w];
          }
        for (int64_t r = 0; r < g.R; ++r) CHECK(seen[r] == 1);
        const int64_t lim = bucket_sweep_limit(g, bi);
        CHECK(lim >= 1 && lim <= INT32_MAX);
        ++shapes;
      }
    g.buckets[bi] = orig;
  }
  retile(g);
  // streams: every bucket on one of at most hw_queues() streams, the launch
  // order a permutation by descending cost, and each bucket, largest first,
  // placed on a stream with the least cost so far
  CHECK(g.n_streams >= 1 && g.n_streams <= 8 && g.n_streams <= (int32_t)g.buckets.size());
  {
    std::vector<int64_t> load(g.n_streams, 0);
    std::vector<int> seen_b(g.buckets.size(), 0);
    for (size_t i = 0; i < g.launch_order.size(); ++i) {
      const int32_t b = g.launch_order[i];
      CHECK(b >= 0 && b < (int32_t)g.buckets.size() && !seen_b[b]);
      seen_b[b] = 1;
      if (i) CHECK(g.bucket_cost[g.launch_order[i - 1]] >= g.bucket_cost[b]);
      CHECK(g.stream_of[b] >= 0 && g.stream_of[b] < g.n_streams);
      int64_t lo = load[0];
      for (int64_t v : load) lo = std::min(lo, v);
      CHECK(load[g.stream_of[b]] == lo);  // placed on a least loaded stream
      load[g.stream_of[b]] += g.bucket_cost[b];
    }
  }
  printf("%s systems %zu bytes %zu buckets %zu streams %d shapes %d sweep_limit %lld pairs_limit %lld\n", name,
         systems.size(), bytes, g.buckets.size(), g.n_streams, shapes, (long long)default_limit,
         (long long)pairs_sweep_limit(g));
}

static void expect_reject(const char *name, const Sys &s, int32_t code) {
  const ising_system_desc d = s.desc();
  size_t bytes = 0;
  const int32_t rc = ising_graph_bytes(&d, 1, &bytes);
  if (rc != code) {
    fprintf(stderr, "%s: rc %d, expected %d (%s)\n", name, rc, code, ising_last_error());
    exit(1);
  }
  printf("reject %s rc %d: %s\n", name, rc, ising_last_error());
}

int main() {
  // workload shapes: the 256-spin ladder, the throughput and many-replica
  // systems, uneven sizes, open slices, random graphs
  check_batch("A", {chimera(2, 8, 16, 1)});
  check_batch("B", {chimera(8, 64, 32, 2), chimera(8, 64, 32, 3)});
  check_batch("C", {chimera(4, 32, 32, 4), chimera(4, 32, 32, 5), chimera(4, 32, 32, 6)});
  {
    std::vector<Sys> d;
    Rng r(4000);
    for (int i = 0; i < 24; ++i) d.push_back(chimera(2 + r.next() % 7, 8 + r.next() % 57, 16 + r.next() % 17, 100 + i));
    check_batch("D", d);
  }
  check_batch("open", {chimera(3, 5, 7, 7, false), chimera(1, 2, 5, 8, false)});
  check_batch("single spin", {random_graph(1, 0, 1, 9)});
  {
    std::vector<Sys> d;
    for (int n = 2; n <= 40; n += 3) d.push_back(random_graph(n, 3 * n, 1 + n % 9, 200 + n));
    check_batch("random graphs", d);
  }
  check_batch("large template", {chimera(8, 3, 2, 11), chimera(7, 4, 3, 12)});

  // invalid descriptions are rejected with their codes, not read out of bounds
  {
    Sys s = chimera(1, 3, 2, 20);
    s.ring = 1;
    s.M = 2;
    expect_reject("ring of two slices", s, ISING_E_RANGE);
  }
  {
    Sys s = chimera(1, 3, 2, 21);
    s.v[0] = s.u[0];
    expect_reject("self edge", s, ISING_E_INVAL);
  }
  {
    Sys s = chimera(1, 3, 2, 22);
    s.v[1] = 8;
    expect_reject("edge out of range", s, ISING_E_INVAL);
  }
  {
    Sys s = chimera(1, 3, 2, 23);
    s.u.push_back(s.u[0]);
    s.v.push_back(s.v[0]);
    s.J.push_back(1);
    expect_reject("duplicate edge", s, ISING_E_INVAL);
  }
  {
    Sys s = random_graph(12, 0, 1, 24);
    for (int j = 1; j <= 9; ++j) s.u.push_back(0), s.v.push_back(j), s.J.push_back(1);
    expect_reject("degree 9", s, ISING_E_RANGE);
  }
  {
    Sys s = chimera(1, 3, 300, 25);
    expect_reject("K above 256", s, ISING_E_RANGE);
  }
  {
    Sys s = chimera(1, 3, 2, 26);
    s.beta[1] = 60.0;
    expect_reject("beta beyond the threshold range", s, ISING_E_RANGE);
  }
  {
    Sys s = chimera(1, 3, 2, 27);
    s.beta[0] = -1.0;
    expect_reject("negative beta", s, ISING_E_RANGE);
  }
  {
    Sys s = chimera(1, 3, 2, 28);
    for (auto &x : s.h) x = 100;
    expect_reject("field bound", s, ISING_E_RANGE);
  }
  {
    Sys s = random_graph(600, 10, 1, 29);
    expect_reject("template above 512 spins", s, ISING_E_RANGE);
  }

  // threshold, acceptance and two-field rows
  Rng r(77);
  std::vector<uint32_t> row(1024), row2(1024);
  for (int i = 0; i < 2000; ++i) {
    const int32_t dmax = r.next() % 64;
    const double beta = (r.next() + 1.0) / 4294967296.0 * 12.0;
    const int32_t rc = ising_threshold_row(beta, dmax, row.data());
    if (2.0 * beta * dmax > 700.0) {
      CHECK(rc == ISING_E_RANGE);
      continue;
    }
    CHECK(rc == ISING_OK && row[0] == 0xffffffffu);
    for (int32_t d = 1; d < dmax; ++d) CHECK(row[d] >= row[d + 1]);
    for (int32_t kind = 1; kind <= 2; ++kind) {
      CHECK(ising_acceptance_row(beta, dmax, kind, row2.data()) == ISING_OK);
      CHECK(row2[0] == 0xffffffffu);
    }
  }
  for (int i = 0; i < 300; ++i) {
    const int32_t ds = r.next() % 20, dt = r.next() % 8;
    const double a = (r.next() % 1000) / 300.0, c = (r.next() % 1000) / 500.0 - 1.0;
    for (int32_t kind = 0; kind <= 2; ++kind) {
      const int32_t rc = ising_two_field_row(a, c, ds, dt, kind, row.data());
      const bool fits = (int64_t)(2 * ds + 1) * (2 * dt + 1) <= 1024;
      if (!fits) CHECK(rc == ISING_E_INVAL);
      else if (2.0 * (fabs(a) * ds + fabs(c) * dt) > 700.0) CHECK(rc == ISING_E_RANGE);
      else CHECK(rc == ISING_OK);
    }
  }
  {
    std::vector<double> b = ladder(32, 0.1, 3.0), wa(32), wc(32);
    CHECK(ising_trotter_weights(b.data(), 32, 64, 1.0, wa.data(), wc.data()) == ISING_OK);
    for (int k = 0; k < 32; ++k) CHECK(wa[k] > 0.0 && isfinite(wc[k]));
  }
  {
    Sys s = chimera(3, 4, 2, 30);
    const ising_system_desc d = s.desc();
    std::vector<int32_t> f(s.S);
    int32_t depth = 0;
    CHECK(ising_level_offsets(&d, f.data(), &depth) == ISING_OK && depth == 6);
  }
  printf("host_check OK\n");
  return 0;
}
