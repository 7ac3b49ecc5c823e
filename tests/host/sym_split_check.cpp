// Host check of the symmetric split (sym_split.hpp): the unit partition,
// the workgroup ranges, the slot lists, and a double-precision replay of the
// products' accumulation order on a random symmetric matrix.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "sym_split.hpp"

using namespace ld;

static int fails = 0;
#define CHECK(c, ...)                                         \
  do {                                                        \
    if (!(c)) {                                               \
      if (fails < 20) {                                       \
        std::printf("FAIL %s:%d: ", __FILE__, __LINE__);      \
        std::printf(__VA_ARGS__);                             \
        std::printf("\n");                                    \
      }                                                       \
      ++fails;                                                \
    }                                                         \
  } while (0)

// the partition: units, costs, workgroup ranges, block coverage, slots
static void check_partition(int64_t n, int ms, int gmax, bool blocks) {
  const SY p = sy_plan(n, 64, ms, gmax);
  // units strip-major: strip S has rows 0 .. me(S) - 1
  int64_t u = 0, cost = 0;
  std::vector<int64_t> before;
  std::vector<int> cover;
  if (blocks) cover.assign((size_t)p.nblk * p.nblk, 0);
  for (int S = 0; S < p.ns; ++S) {
    CHECK(sy_u0(p, S) == u, "u0(%d) = %lld, expected %lld", S, (long long)sy_u0(p, S), (long long)u);
    const int mS = ms * S, me = sy_me(p, S);
    for (int I = 0; I < me; ++I, ++u) {
      CHECK(sy_strip(p, u) == S, "strip(%lld)", (long long)u);
      CHECK(sy_cost_before(p, u) == cost, "cost_before(%lld) = %lld, expected %lld", (long long)u,
            (long long)sy_cost_before(p, u), (long long)cost);
      before.push_back(cost);
      for (int J = (I > mS ? I : mS); J < me; ++J) {
        ++cost;
        if (blocks) ++cover[(size_t)I * p.nblk + J];
      }
    }
  }
  CHECK(u == p.units, "units %lld vs %lld", (long long)u, (long long)p.units);
  CHECK(cost == p.cost, "cost %lld vs %lld", (long long)cost, (long long)p.cost);
  CHECK(sy_cost_before(p, p.units) == p.cost, "cost_before(units)");
  if (blocks)
    for (int I = 0; I < p.nblk; ++I)
      for (int J = 0; J < p.nblk; ++J)
        CHECK(cover[(size_t)I * p.nblk + J] == (J >= I ? 1 : 0), "block (%d, %d) covered %d times", I,
              J, cover[(size_t)I * p.nblk + J]);
  // workgroup ranges: contiguous, in order, covering every unit, balanced
  CHECK(sy_start(p, 0) == 0 && sy_start(p, p.G) == p.units, "range ends");
  int Jt = 1;
  const int64_t per = p.cost / p.G;
  for (int g = 0; g < p.G; ++g) {
    const int64_t a = sy_start(p, g), b = sy_start(p, g + 1);
    CHECK(a <= b, "range %d", g);
    if (a < b) {
      CHECK(sy_wg(p, a) == g && sy_wg(p, b - 1) == g, "wg of range %d", g);
      const int span = sy_strip(p, b - 1) - sy_strip(p, a) + 1;
      if (span > Jt) Jt = span;
      const int64_t c = sy_cost_before(p, b) - sy_cost_before(p, a);
      CHECK(c <= per + 2 * ms, "workgroup %d cost %lld vs %lld", g, (long long)c, (long long)per);
    }
  }
  CHECK(Jt == p.Jt, "Jt %d vs %d", Jt, p.Jt);
  // transposed lists: the distinct workgroups owning units (R / ms, I < R)
  for (int R = 0; R < p.nblk; ++R) {
    const int SR = R / ms;
    std::vector<int64_t> want;
    int last = -1;
    for (int I = 0; I < R; ++I) {
      const int g = sy_wg(p, sy_u0(p, SR) + I);
      if (g != last) {
        want.push_back(sy_tr_slot(p, g, sy_strip(p, sy_start(p, g)), SR, R));
        last = g;
      }
    }
    std::vector<int64_t> got(want.size() + 4);
    const int cnt = sy_tr_list(p, R, got.data(), (int)got.size());
    CHECK(cnt == (int)want.size(), "R %d list %d vs %zu", R, cnt, want.size());
    for (int k = 0; k < cnt && k < (int)want.size(); ++k) CHECK(got[k] == want[k], "R %d slot %d", R, k);
  }
}

// the products' accumulation (direct per unit, transposed per workgroup and
// strip, then the epilogue's sums) against a dense product
static void check_replay(int64_t n, int ms, int gmax, int s, uint64_t seed) {
  const SY p = sy_plan(n, s, ms, gmax);
  const int64_t N = (int64_t)p.nblk * 128;  // padded: rows >= n of V are zero
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::vector<double> M((size_t)N * N, 0.0), V((size_t)N * s, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i; j < n; ++j) M[(size_t)i * N + j] = M[(size_t)j * N + i] = U(rng);
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < s; ++c) V[(size_t)i * s + c] = U(rng);
  const int64_t TILE = 128 * (int64_t)s;
  const int64_t slots = p.units + (int64_t)p.G * p.Jt * ms;
  std::vector<double> part((size_t)(slots * TILE), 0.0);
  std::vector<char> written((size_t)slots, 0);
  for (int g = 0; g < p.G; ++g) {
    int64_t u = sy_start(p, g);
    const int64_t ue = sy_start(p, g + 1);
    if (u >= ue) continue;
    const int Sf = sy_strip(p, u);
    std::vector<double> accT((size_t)ms * TILE, 0.0);
    int S = Sf, I = (int)(u - sy_u0(p, Sf));
    auto flush = [&](int Sx) {
      for (int b = 0; b < ms; ++b) {
        const int64_t sl = sy_tr_slot(p, g, Sf, Sx, ms * Sx + b);
        CHECK(sl >= p.units && sl < slots, "transposed slot range");
        written[(size_t)sl] = 1;
        for (int64_t e = 0; e < TILE; ++e) part[(size_t)(sl * TILE + e)] = accT[(size_t)(b * TILE + e)];
      }
      std::fill(accT.begin(), accT.end(), 0.0);
    };
    while (true) {
      const int mS = ms * S, me = sy_me(p, S);
      std::vector<double> acc((size_t)TILE, 0.0);
      for (int J = (I > mS ? I : mS); J < me; ++J)
        for (int r = 0; r < 128; ++r)
          for (int k = 0; k < 128; ++k) {
            const double m = M[(size_t)(128 * I + r) * N + 128 * J + k];
            for (int c = 0; c < s; ++c) {
              acc[(size_t)r * s + c] += m * V[(size_t)(128 * J + k) * s + c];
              if (J > I) accT[(size_t)((J - mS) * TILE + k * s + c)] += m * V[(size_t)(128 * I + r) * s + c];
            }
          }
      const int64_t sl = sy_dir_slot(p, S, I);
      CHECK(sl >= 0 && sl < p.units, "direct slot range");
      CHECK(!written[(size_t)sl], "direct slot written twice");
      written[(size_t)sl] = 1;
      for (int64_t e = 0; e < TILE; ++e) part[(size_t)(sl * TILE + e)] = acc[(size_t)e];
      ++u;
      int Sn = S, In = I + 1;
      if (In >= me) {
        Sn = S + 1;
        In = 0;
      }
      if (u >= ue) break;
      if (Sn != S) flush(S);
      S = Sn;
      I = In;
    }
    flush(S);
  }
  double err = 0.0, ref = 0.0;
  for (int R = 0; R < p.nblk; ++R) {
    const int SR = R / ms;
    std::vector<int64_t> list;
    for (int S = SR; S < p.ns; ++S) {
      list.push_back(sy_dir_slot(p, S, R));
      CHECK(sy_dir_slot(p, S, R) == sy_dir_base(p, R) + (S - SR), "direct slots of R contiguous");
    }
    std::vector<int64_t> tr(64);
    const int cnt = sy_tr_list(p, R, tr.data(), 64);
    CHECK(cnt <= 64, "list length");
    for (int k = 0; k < cnt && k < 64; ++k) list.push_back(tr[k]);
    for (int64_t sl : list) CHECK(written[(size_t)sl], "R %d reads unwritten slot %lld", R, (long long)sl);
    for (int r = 0; r < 128; ++r) {
      const int64_t i = 128 * (int64_t)R + r;
      if (i >= n) break;
      for (int c = 0; c < s; ++c) {
        double y = 0.0;
        for (int64_t sl : list) y += part[(size_t)(sl * TILE + r * s + c)];
        double want = 0.0;
        for (int64_t k = 0; k < n; ++k) want += M[(size_t)i * N + k] * V[(size_t)k * s + c];
        err = std::max(err, std::abs(y - want));
        ref = std::max(ref, std::abs(want));
      }
    }
  }
  CHECK(err <= 1e-12 * ref, "replay n=%lld ms=%d G=%d: max error %.3g of %.3g", (long long)n, ms, p.G, err,
        ref);
}

int main() {
  // partitions: tiny, ragged, several strips per workgroup, the solver sizes
  const int64_t sizes[] = {1, 127, 128, 129, 1000, 2000, 4097, 16384, 20000, 50000, 100000, 200000};
  for (int64_t n : sizes)
    for (int ms : {1, 2, 3, 4})
      for (int gmax : {1, 3, 8, 512}) check_partition(n, ms, gmax, n <= 50000);
  // replays: ragged n, workgroups that span strips and strips split over workgroups
  check_replay(1701, 2, 7, 8, 1);
  check_replay(1701, 2, 1, 8, 2);
  check_replay(2000, 3, 5, 4, 3);
  check_replay(129, 2, 3, 4, 4);
  check_replay(3100, 2, 512, 3, 5);
  if (fails) {
    std::printf("%d failures\n", fails);
    return 1;
  }
  std::printf("OK\n");
  return 0;
}
