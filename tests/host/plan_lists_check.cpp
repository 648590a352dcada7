// Host-side check of the plan's point lists (no GPU): for a few grids and
// split parts, every kept data sample and every Radon sample is owned by
// exactly one band, in index order, at a row inside that band; every
// sample sits in the spread list of each band its 4 x 4 stencil reaches and
// of no other; chunks tile the lists band by band within their size limits;
// a spread chunk's column range holds every stencil of its entries, stays
// within the accumulator's width and the window, and its partial rows follow
// the previous chunk's; the Radon entries of one slowness share their angle
// coordinate and weight.  Grids with band heights 8, 4 and 2 are covered,
// and 24 seeded random grids.
// Prints "ok" and exits 0, or prints the first failure and exits 1.
#include <cmath>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace hrt;

static int fails = 0;
#define CHECK(cond, ...)                        \
  do {                                          \
    if (!(cond)) {                              \
      std::printf(__VA_ARGS__);                 \
      std::printf("\n");                        \
      ++fails;                                  \
      return;                                   \
    }                                           \
  } while (0)

// absolute lattice row of an entry of band b's list
static double entry_row(const Geometry& g, int b, const PointEntry& e) {
  return g.u0 + b * g.R - 2 + std::ldexp(static_cast<double>(e.yq), -kYFracBits);
}

static void check_chunks(const BandLists& L, int nb, int max_entries, const char* what) {
  CHECK(L.off.size() == static_cast<size_t>(nb) + 1, "%s: band offsets", what);
  CHECK(L.chunk_off.front() == 0 && L.chunk_off.back() == L.off[nb], "%s: chunk ends", what);
  CHECK(L.band_chunk.size() == static_cast<size_t>(nb) + 1, "%s: band chunks", what);
  for (size_t c = 0; c + 1 < L.chunk_off.size(); ++c) {
    const int b = L.chunk_band[c];
    CHECK(L.chunk_off[c] <= L.chunk_off[c + 1], "%s: chunk %zu order", what, c);
    CHECK(L.chunk_off[c + 1] - L.chunk_off[c] <= max_entries, "%s: chunk %zu size", what, c);
    CHECK(L.off[b] <= L.chunk_off[c] && L.chunk_off[c + 1] <= L.off[b + 1],
          "%s: chunk %zu outside band %d", what, c, b);
    CHECK(L.band_chunk[b] <= static_cast<int>(c) && static_cast<int>(c) < L.band_chunk[b + 1],
          "%s: band_chunk of chunk %zu", what, c);
  }
}

static void check_spans(const Geometry& g, const BandLists& L, const char* what) {
  const size_t nc = L.chunk_band.size();
  CHECK(L.chunk_col.size() == 2 * nc && L.chunk_hp.size() == nc, "%s: span tables", what);
  int64_t hp = 0;
  for (size_t c = 0; c < nc; ++c) {
    const int lo = L.chunk_col[2 * c], wc = L.chunk_col[2 * c + 1];
    CHECK(lo % 4 == 0 && wc % 4 == 0 && lo >= 0 && wc >= 0, "%s: chunk %zu columns", what, c);
    CHECK(wc <= g.spread_cols && lo + wc <= g.W, "%s: chunk %zu spans %d columns from %d",
          what, c, wc, lo);
    CHECK(L.chunk_hp[c] == hp, "%s: chunk %zu partial at %lld, want %lld", what, c,
          static_cast<long long>(L.chunk_hp[c]), static_cast<long long>(hp));
    hp += static_cast<int64_t>(g.R) * wc;
    CHECK(L.chunk_off[c + 1] == L.chunk_off[c] || wc > 0, "%s: chunk %zu empty span", what, c);
    for (int64_t i = L.chunk_off[c]; i < L.chunk_off[c + 1]; ++i) {
      const int cx = static_cast<int>(L.e[i].xq >> g.x_frac_bits) - 1;
      CHECK(cx >= lo && cx + 4 <= lo + wc, "%s: chunk %zu entry %lld taps %d..%d outside %d..%d",
            what, c, static_cast<long long>(i), cx, cx + 3, lo, lo + wc - 1);
    }
  }
  CHECK(L.hp_floats == hp, "%s: partial floats %lld, want %lld", what,
        static_cast<long long>(L.hp_floats), static_cast<long long>(hp));
  CHECK(static_cast<int64_t>(g.R) * g.spread_cols * 8 <= g.spread_bytes,
        "%s: spread LDS", what);
}

// `expected`: the indices the point set must hold, in increasing order
static void check_set(const Geometry& g, const BandLists& spread, const BandLists& own,
                      const std::vector<uint32_t>& expected, const char* what) {
  const int nb = g.nbands;
  check_chunks(spread, nb, g.spread_chunk, what);
  check_chunks(own, nb, g.gather_chunk, what);
  check_spans(g, spread, what);
  if (fails) return;
  // owned: each expected index once, band-major, increasing inside a band,
  // its row floor inside the band (a row within 2^-20 of an integer may
  // round to either side)
  std::map<uint32_t, double> row_of;
  for (int b = 0; b < nb; ++b) {
    uint32_t prev = 0;
    for (int64_t i = own.off[b]; i < own.off[b + 1]; ++i) {
      const PointEntry& e = own.e[i];
      CHECK(i == own.off[b] || e.idx > prev, "%s: own band %d not increasing", what, b);
      prev = e.idx;
      const double y = entry_row(g, b, e);
      const int lo = g.u0 + b * g.R, hi = std::min(lo + g.R, g.u1);
      const double fy = std::floor(y + 1e-6), fy2 = std::floor(y - 1e-6);
      CHECK((fy >= lo && fy < hi) || (fy2 >= lo && fy2 < hi),
            "%s: own entry %u row %.6f outside band %d [%d, %d)", what, e.idx, y, b, lo, hi);
      CHECK(row_of.emplace(e.idx, y).second, "%s: sample %u owned twice", what, e.idx);
      const double x = std::ldexp(static_cast<double>(e.xq), -g.x_frac_bits);
      CHECK(x >= 1.0 - 1e-6 && x + 3.0 < g.W + 1e-6, "%s: column %.4f outside window", what, x);
    }
  }
  CHECK(row_of.size() == expected.size(), "%s: %zu owned, %zu expected", what, row_of.size(),
        expected.size());
  for (uint32_t idx : expected) CHECK(row_of.count(idx), "%s: sample %u not owned", what, idx);
  // spread: entry in band b iff the stencil rows floor(y)-1 .. floor(y)+2
  // meet the band's rows; the same row as the owner's
  std::map<uint32_t, int> seen;
  for (int b = 0; b < nb; ++b) {
    const int lo = g.u0 + b * g.R, hi = std::min(lo + g.R, g.u1);
    for (int64_t i = spread.off[b]; i < spread.off[b + 1]; ++i) {
      const PointEntry& e = spread.e[i];
      const double y = entry_row(g, b, e);
      CHECK(row_of.count(e.idx), "%s: spread entry %u not a sample", what, e.idx);
      CHECK(std::fabs(y - row_of[e.idx]) < 1e-6, "%s: sample %u rows differ", what, e.idx);
      const int iy = static_cast<int>(std::floor(y + 1e-9));
      CHECK(iy + 2 >= lo - 1 && iy - 1 <= hi, "%s: sample %u in band %d it cannot reach", what,
            e.idx, b);
      ++seen[e.idx];
    }
  }
  for (const auto& kv : row_of) {
    const int iy = static_cast<int>(std::floor(kv.second));
    int want = 0;
    for (int b = 0; b < nb; ++b) {
      const int lo = g.u0 + b * g.R, hi = std::min(lo + g.R, g.u1);
      if (iy - 1 < hi && iy + 2 >= lo) ++want;
    }
    const int got = seen.count(kv.first) ? seen[kv.first] : 0;
    // a row within rounding of an integer may reach one band more or less
    CHECK(std::abs(got - want) <= 1 && got >= 1, "%s: sample %u in %d spread lists, want %d",
          what, kv.first, got, want);
  }
}

// Radon entries travel to the device without their angle coordinate and
// weight, which are taken from a per-slowness table: every Radon entry of
// one slowness (in both lists) must carry the same pair, and the slowness
// row of an index, (idx * m) >> s with s = 32 + ceil(log2 ld) and
// m = ceil(2^s / ld), must be idx / ld exactly.
static void check_radon_slowness(const Geometry& g, const BandLists& spread,
                                 const BandLists& own, const char* what) {
  const PartView& v = g.view;
  const uint64_t ld = static_cast<uint64_t>(v.radon_ld);
  int lg = 0;
  while ((uint64_t{1} << lg) < ld) ++lg;
  const int sh = 32 + lg;
  const uint64_t m = ((uint64_t{1} << sh) + ld - 1) / ld;
  std::map<int, std::pair<uint32_t, float>> pair;
  for (const BandLists* L : {&spread, &own})
    for (const PointEntry& e : L->e) {
      const uint64_t row = e.idx / ld;
      CHECK(((static_cast<uint64_t>(e.idx) * m) >> sh) == row,
            "%s: index %u: multiply-shift row differs", what, e.idx);
      const int l = static_cast<int>(row) - v.radon_row0;
      CHECK(l >= 0 && l < g.d.nq, "%s: index %u outside the plan's slownesses", what, e.idx);
      auto it = pair.find(l);
      if (it == pair.end()) {
        pair[l] = {e.xq, e.w};
      } else {
        CHECK(it->second.first == e.xq && it->second.second == e.w,
              "%s: slowness %d: entries disagree on angle or weight", what, l);
      }
    }
}

static void run(const char* name, const hrt_desc& d, const PartView* view, int want_R = 0) {
  Geometry g;
  std::string err;
  if (build_geometry(d, 163840 - 4096, g, err, view) != HRT_OK) {
    std::printf("%s: geometry: %s\n", name, err.c_str());
    ++fails;
    return;
  }
  if (want_R && g.R != want_R) {
    std::printf("%s: band height %d, want %d\n", name, g.R, want_R);
    ++fails;
    return;
  }
  PointTables t;
  if (build_point_tables(g, t, err) != HRT_OK) {
    std::printf("%s: tables: %s\n", name, err.c_str());
    ++fails;
    return;
  }
  const PartView& v = g.view;
  std::vector<uint32_t> data, radon;
  for (int k = 0; k < d.nx; ++k)
    for (int j = std::max(g.jmin[k], v.j_lo); j < v.j_hi; ++j)
      data.push_back(static_cast<uint32_t>(k * v.data_ld + j));
  for (int l = 0; l < d.nq; ++l)
    for (int i = 0; i < d.ntau; ++i)
      radon.push_back(static_cast<uint32_t>((v.radon_row0 + l) * v.radon_ld + i));
  if (static_cast<int64_t>(data.size()) != g.n_kept) {
    std::printf("%s: n_kept %lld, %zu expected\n", name, static_cast<long long>(g.n_kept),
                data.size());
    ++fails;
  }
  std::string a = std::string(name) + " data", b = std::string(name) + " radon";
  check_set(g, t.data_spread, t.data_own, data, a.c_str());
  check_set(g, t.radon_spread, t.radon_own, radon, b.c_str());
  check_radon_slowness(g, t.radon_spread, t.radon_own, b.c_str());
  if (!(t.cmax_data > 0 && t.cmax_radon > 0)) {
    std::printf("%s: cmax\n", name);
    ++fails;
  }
}

// splitmix64: a seeded stream of 64-bit values for the random grids
static uint64_t rng_state = 0x2026;
static uint64_t next_u64() {
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double uniform(double lo, double hi) {
  return lo + (hi - lo) * static_cast<double>(next_u64() >> 11) * 0x1.0p-53;
}
static int uniform_int(int lo, int hi) {  // [lo, hi)
  return lo + static_cast<int>(next_u64() % static_cast<uint64_t>(hi - lo));
}

// Seeded random grids (sizes, steps, offsets, slowness ranges, oversampling
// and the band/chunk variants all drawn at random); a grid the geometry
// rejects is drawn again.
static void run_random(int count) {
  const uint32_t variants[] = {0u, HRT_TUNE_SPREAD_HALF, HRT_TUNE_GATHER_DOUBLE,
                               HRT_TUNE_BAND4 | HRT_TUNE_SPREAD_HALF, HRT_TUNE_BAND2};
  const double ovs[] = {1.5, 2.0, 2.5, 3.0};
  const double dts[] = {0.002, 0.004, 0.008};
  int done = 0;
  while (done < count) {
    hrt_desc d{};
    d.nt = uniform_int(4, 600);
    d.nx = uniform_int(4, 200);
    d.dt = dts[uniform_int(0, 3)];
    d.x0 = uniform_int(0, 2) ? 0.0 : uniform(0.0, 0.3);
    const double X = uniform(0.2, 4.0);
    if (X <= d.x0 + 0.05) continue;
    d.dx = (X - d.x0) / (d.nx - 1);
    const double T = (d.nt - 1) * d.dt;
    d.ntau = uniform_int(4, 600);
    d.tau0 = uniform_int(0, 2) ? 0.0 : uniform(0.0, 0.2 * T);
    d.dtau = (T - d.tau0) / (d.ntau - 1) * uniform(0.5, 1.0);
    d.nq = uniform_int(4, 200);
    d.q0 = uniform(0.0, 0.4);
    d.dq = (uniform(d.q0 + 0.05, 1.0) - d.q0) / (d.nq - 1);
    d.oversample = ovs[uniform_int(0, 4)];
    d.flags = variants[uniform_int(0, 5)];
    Geometry g;
    std::string err;
    if (build_geometry(d, 163840 - 4096, g, err, nullptr) != HRT_OK) continue;
    run(("random " + std::to_string(done)).c_str(), d, nullptr);
    ++done;
  }
}

int main() {
  const double qmin = 0.25, qmax = 1.0 / 1.5;
  hrt_desc c1{256, 128, 0.004, 0.0, 2.0 / 127, 256, 128, 0.0, 0.004, qmin,
              (qmax - qmin) / 127, 2.0, 0};
  hrt_desc odd{37, 23, 0.01, 0.05, 0.03, 29, 19, 0.07, 0.01, 0.3, 0.021, 2.5, 0};
  hrt_desc ragged{301, 77, 0.004, 0.1, 0.025, 250, 61, 0.05, 0.0045, 0.22, 0.0075, 2.0, 0};
  run("c1", c1, nullptr, 8);
  run("odd", odd, nullptr);
  run("ragged", ragged, nullptr, 8);
  // band heights 4 and 2, and the other chunk sizes
  for (const hrt_desc* base : {&c1, &ragged}) {
    hrt_desc d = *base;
    d.flags = HRT_TUNE_BAND4 | HRT_TUNE_SPREAD_HALF;
    run(base == &c1 ? "c1 band4" : "ragged band4", d, nullptr, 4);
    d.flags = HRT_TUNE_BAND2 | HRT_TUNE_GATHER_DOUBLE;
    run(base == &c1 ? "c1 band2" : "ragged band2", d, nullptr, 2);
  }
  // the parts of two splits
  const int32_t te[] = {0, 96, 256}, qe[] = {0, 64, 128};
  const int32_t te2[] = {0, 120, 301}, qe2[] = {0, 20, 41, 61};
  for (int p = 0; p < 4; ++p) {
    hrt_desc sub;
    PartView v;
    std::string err;
    if (split_part(c1, 2, te, 2, qe, p, sub, v, err) != HRT_OK) {
      std::printf("c1 part %d: %s\n", p, err.c_str());
      ++fails;
      continue;
    }
    run(("c1 part " + std::to_string(p)).c_str(), sub, &v);
  }
  for (int p = 0; p < 6; ++p) {
    hrt_desc sub;
    PartView v;
    std::string err;
    if (split_part(ragged, 2, te2, 3, qe2, p, sub, v, err) != HRT_OK) {
      std::printf("ragged part %d: %s\n", p, err.c_str());
      ++fails;
      continue;
    }
    run(("ragged part " + std::to_string(p)).c_str(), sub, &v);
  }
  run_random(24);
  if (fails) return 1;
  std::printf("ok\n");
  return 0;
}
