// Host-side input checks of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer: well-formed inputs pass, each malformed case is
// rejected with a message, and random malformed arrays of the documented
// sizes are rejected or accepted without any out-of-bounds access.  Exits 0
// when every expectation holds (a sanitizer report aborts the run).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "validate.hpp"

static int failures = 0;
#define EXPECT(cond, what)                                         \
  do {                                                             \
    if (!(cond)) { std::printf("FAILED: %s\n", what); ++failures; } \
  } while (0)

struct Csr { int32_t n; std::vector<int32_t> rp, col; };

static Csr grid(int a, int b) {
  Csr g;
  g.n = a * b;
  std::vector<std::vector<int32_t>> adj(g.n);
  for (int i = 0; i < a; ++i)
    for (int j = 0; j < b; ++j) {
      const int v = i * b + j;
      if (j + 1 < b) { adj[v].push_back(v + 1); adj[v + 1].push_back(v); }
      if (i + 1 < a) { adj[v].push_back(v + b); adj[v + b].push_back(v); }
    }
  g.rp.push_back(0);
  for (auto& r : adj) {
    std::sort(r.begin(), r.end());
    for (int v : r) g.col.push_back(v);
    g.rp.push_back((int32_t)g.col.size());
  }
  return g;
}

static bool graph_ok(const Csr& g, const int32_t* c = nullptr, const int32_t* w = nullptr) {
  char msg[256];
  return mm::check_graph(g.n, (int64_t)g.col.size(), g.rp.data(), g.col.data(), c, w, msg,
                         sizeof(msg));
}

// path 0-1-2, k = 2: row 0 = [1 | 2], row 1 = [0, 2 | ], row 2 = [1 | 0]
struct Set { int32_t n, k; std::vector<int64_t> off; std::vector<int32_t> hend, nbr; };
static Set path3() {
  return {3, 2, {0, 2, 4, 6}, {1, 2, 2, 2, 1, 2}, {1, 2, 0, 2, 1, 0}};
}
static bool set_ok(const Set& s) {
  char msg[256];
  return mm::check_stress_set(s.n, s.k, s.off.data(), s.hend.data(),
                              s.nbr.empty() ? nullptr : s.nbr.data(), msg, sizeof(msg));
}

int main() {
  // graphs
  Csr g = grid(7, 5);
  EXPECT(graph_ok(g), "grid accepted");
  std::vector<int32_t> c(g.n, 2), w(g.col.size(), 3);
  EXPECT(graph_ok(g, c.data(), w.data()), "weighted grid accepted");
  { Csr h = g; h.col[3] = g.n; EXPECT(!graph_ok(h), "column out of range"); }
  { Csr h = g; h.col[0] = 0; EXPECT(!graph_ok(h), "self-loop"); }
  { Csr h = g; std::swap(h.col[0], h.col[1]); EXPECT(!graph_ok(h), "unsorted row"); }
  { Csr h = g; h.rp[3] = h.rp[2] - 1; EXPECT(!graph_ok(h), "row_ptr decreasing"); }
  { Csr h = g; h.rp.back() -= 1; EXPECT(!graph_ok(h), "row_ptr[n] != nnz"); }
  { std::vector<int32_t> w2 = w; w2[0] = 5; EXPECT(!graph_ok(g, nullptr, w2.data()), "asymmetric weight"); }
  { std::vector<int32_t> c2 = c; c2[4] = 0; EXPECT(!graph_ok(g, c2.data()), "node weight 0"); }
  { Csr one; one.n = 1; one.rp = {0, 0}; EXPECT(!graph_ok(one), "n = 1"); }
  // stress sets
  EXPECT(set_ok(path3()), "path set accepted");
  { Set s = path3(); s.nbr[1] = 3; EXPECT(!set_ok(s), "id out of range"); }
  { Set s = path3(); s.nbr[1] = 0; EXPECT(!set_ok(s), "row holds itself"); }
  { Set s = path3(); s.hend[0] = 2; s.hend[1] = 2; EXPECT(!set_ok(s), "missing mirror"); }
  { Set s = {3, 1, {0, 1, 2, 2}, {1, 1, 0}, {1, 0}}; EXPECT(!set_ok(s), "empty row"); }
  // random arrays of the documented sizes: accepted or rejected, never read
  // out of bounds
  std::mt19937_64 rng(12345);
  int accepted = 0;
  for (int it = 0; it < 20000; ++it) {
    const int32_t n = 2 + (int32_t)(rng() % 6), k = 1 + (int32_t)(rng() % 3);
    Set s{n, k, std::vector<int64_t>(n + 1), std::vector<int32_t>((size_t)n * k), {}};
    int64_t o = 0;
    s.off[0] = (rng() % 16) ? 0 : (int64_t)(rng() % 3);
    for (int32_t u = 0; u < n; ++u) {
      const int64_t len = (int64_t)(rng() % (size_t)(n + 1)) - ((rng() % 12) ? 0 : 2);
      o = (u == 0 ? s.off[0] : o) + len;
      s.off[u + 1] = o;
      int32_t run = 0;
      for (int32_t h = 0; h < k; ++h) {
        run += (int32_t)(rng() % 3);
        s.hend[(size_t)u * k + h] = (h == k - 1 && (rng() % 4)) ? (int32_t)std::max<int64_t>(len, 0) : run;
      }
    }
    if (s.off[n] < 0) s.off[n] = 0;
    s.nbr.resize((size_t)std::max<int64_t>(s.off[n], 0));
    for (auto& v : s.nbr) v = (int32_t)(rng() % (size_t)(n + 1)) - ((rng() % 20) ? 0 : 1);
    accepted += set_ok(s) ? 1 : 0;
  }
  for (int it = 0; it < 20000; ++it) {
    Csr h;
    h.n = 2 + (int32_t)(rng() % 6);
    h.rp.assign(h.n + 1, 0);
    for (int32_t u = 0; u < h.n; ++u) h.rp[u + 1] = h.rp[u] + (int32_t)(rng() % 4) - ((rng() % 10) ? 0 : 1);
    if (h.rp[h.n] < 0) h.rp[h.n] = 0;
    h.col.resize((size_t)h.rp[h.n]);
    for (auto& v : h.col) v = (int32_t)(rng() % (size_t)(h.n + 1)) - ((rng() % 20) ? 0 : 1);
    accepted += graph_ok(h) ? 1 : 0;
  }
  // tune records
  const int64_t good[7] = {1, 1000, 50000, 2, 12, 64, 4};
  EXPECT(mm::check_tune_record(good, 64), "tune record accepted");
  int64_t badr[7];
  std::memcpy(badr, good, sizeof(good)); badr[4] = 14; EXPECT(!mm::check_tune_record(badr, 64), "tile bits");
  std::memcpy(badr, good, sizeof(good)); badr[5] = 3; EXPECT(!mm::check_tune_record(badr, 64), "lanes");
  std::memcpy(badr, good, sizeof(good)); badr[6] = 3; EXPECT(!mm::check_tune_record(badr, 64), "blocks");
  std::printf("random inputs accepted: %d of 40000; failures: %d\n", accepted, failures);
  return failures ? 1 : 0;
}
