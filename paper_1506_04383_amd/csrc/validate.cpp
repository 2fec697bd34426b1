// Host-side input checks of the C-ABI (see validate.hpp).
#include "validate.hpp"

#include <algorithm>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <vector>

namespace mm {
namespace {

bool bad(char* msg, size_t cap, const char* fmt, ...) {
  if (msg && cap > 0) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, cap, fmt, ap);
    va_end(ap);
  }
  return false;
}

}  // namespace

bool check_graph(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col, const int32_t* c,
                 const int32_t* w, char* msg, size_t cap) {
  if (n < 2) return bad(msg, cap, "graph needs at least 2 vertices (n=%d)", n);
  if (!rp || (nnz > 0 && !col)) return bad(msg, cap, "NULL graph array");
  if (rp[0] != 0 || (int64_t)rp[n] != nnz) return bad(msg, cap, "row_ptr[0] must be 0 and row_ptr[n] == nnz");
  for (int32_t u = 0; u < n; ++u)
    if (rp[u + 1] < rp[u]) return bad(msg, cap, "row_ptr not monotone at %d", u);
  for (int32_t u = 0; u < n; ++u) {
    if (rp[u + 1] == rp[u]) return bad(msg, cap, "vertex %d is isolated (rho_u = 0)", u);
    if (c && c[u] < 1) return bad(msg, cap, "node weight of %d < 1", u);
    for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
      const int32_t v = col[e];
      if (v < 0 || v >= n) return bad(msg, cap, "column %d out of range in row %d", v, u);
      if (v == u) return bad(msg, cap, "self-loop at %d", u);
      if (e > rp[u] && col[e - 1] >= v) return bad(msg, cap, "row %d not strictly ascending", u);
      if (w && w[e] < 1) return bad(msg, cap, "edge weight < 1 in row %d", u);
    }
  }
  for (int32_t u = 0; u < n; ++u) {
    for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
      const int32_t v = col[e];
      const int32_t* b = col + rp[v];
      const int32_t* en = col + rp[v + 1];
      const int32_t* it = std::lower_bound(b, en, u);
      if (it == en || *it != u) return bad(msg, cap, "edge %d-%d has no reverse", u, v);
      if (w && w[it - col] != w[e]) return bad(msg, cap, "edge weights of %d-%d differ", u, v);
    }
  }
  return true;
}

bool check_stress_set(int32_t n, int32_t k, const int64_t* off, const int32_t* hend,
                      const int32_t* nbr, char* msg, size_t cap) {
  if (!off || !hend) return bad(msg, cap, "NULL argument");
  if (n < 2) return bad(msg, cap, "n < 2");
  if (k < 1 || k > 8) return bad(msg, cap, "k must be in [1, 8]");
  if (off[0] != 0) return bad(msg, cap, "off[0] = %lld, must be 0", (long long)off[0]);
  for (int32_t u = 0; u < n; ++u) {
    const int64_t len = off[u + 1] - off[u];
    if (len < 0) return bad(msg, cap, "off decreases at row %d", u);
    // Eq. 2 divides by rho_u = sum of w_uv over S(u): an empty row has none
    if (len == 0) return bad(msg, cap, "row %d is empty (rho_u = 0 in Eq. 2)", u);
    if (len >= n) return bad(msg, cap, "row %d has %lld entries (at most n-1)", u, (long long)len);
    int32_t prev = 0;
    for (int32_t h = 0; h < k; ++h) {
      const int32_t e = hend[(size_t)u * k + h];
      if (e < prev) return bad(msg, cap, "hend of row %d decreases at distance %d", u, h + 1);
      prev = e;
    }
    if (prev != len)
      return bad(msg, cap, "hend of row %d ends at %d, row has %lld entries", u, prev, (long long)len);
  }
  const int64_t total = off[n];
  if (total > 0 && !nbr) return bad(msg, cap, "nbr is NULL");
  std::vector<int32_t> seen((size_t)n, -1);
  for (int32_t u = 0; u < n; ++u) {
    const int32_t* row = nbr + off[u];
    int32_t s0 = 0;
    for (int32_t h = 0; h < k; ++h) {
      const int32_t s1 = hend[(size_t)u * k + h];
      for (int32_t i = s0; i < s1; ++i) {
        const int32_t v = row[i];
        if (v < 0 || v >= n) return bad(msg, cap, "row %d: id %d out of range", u, v);
        if (v == u) return bad(msg, cap, "row %d holds itself", u);
        if (i > s0 && row[i - 1] >= v)
          return bad(msg, cap, "row %d: ids at distance %d not strictly increasing", u, h + 1);
        if (seen[(size_t)v] == u) return bad(msg, cap, "row %d holds %d twice", u, v);
        seen[(size_t)v] = u;
      }
      s0 = s1;
    }
  }
  // every row is well formed now: look up the mirror of each pair, u in the
  // group of row v with the same distance
  for (int32_t u = 0; u < n; ++u) {
    const int32_t* row = nbr + off[u];
    int32_t s0 = 0;
    for (int32_t h = 0; h < k; ++h) {
      const int32_t s1 = hend[(size_t)u * k + h];
      for (int32_t i = s0; i < s1; ++i) {
        const int32_t v = row[i];
        const int32_t* vr = nbr + off[v];
        const int32_t* b = vr + (h ? hend[(size_t)v * k + h - 1] : 0);
        const int32_t* e = vr + hend[(size_t)v * k + h];
        const int32_t* f = std::lower_bound(b, e, u);
        if (f == e || *f != u)
          return bad(msg, cap, "pair (%d, %d) at distance %d has no mirror (%d, %d)", u, v, h + 1, v, u);
      }
      s0 = s1;
    }
  }
  return true;
}

bool check_tune_record(const int64_t* r, int32_t sliced_code) {
  const bool tb_ok = r[4] == 0 || (r[4] >= 11 && r[4] <= 13);
  const bool g_ok = r[5] >= 1 && r[5] <= 64 && (r[5] & (r[5] - 1)) == 0 &&
                    (r[4] == 0 ? r[5] >= 8 : (r[5] <= 16 || r[5] == sliced_code));
  const bool nb_ok = r[4] == 0 ? r[6] == 0 : (r[6] == 0 || r[6] == 2 || r[6] == 4);
  return tb_ok && g_ok && nb_ok && (r[0] == 0 || r[0] == 1) && r[1] >= 0 && r[1] <= INT32_MAX &&
         r[2] >= 0 && r[3] >= 1 && r[3] <= INT32_MAX;
}

}  // namespace mm
