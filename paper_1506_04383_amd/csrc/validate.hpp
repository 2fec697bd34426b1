// Host-side input checks of the C-ABI, in plain C++ (no HIP): the library
// compiles them with the rest of its host code, and a CPU test builds them
// with g++ under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Each check returns true when the input is well formed; otherwise false
// with a description of the first violation in msg (at most cap bytes,
// NUL-terminated).  Every array is read only within the bounds that the
// checks before have established, so malformed input never leads to an
// out-of-bounds read.
#pragma once
#include <cstddef>
#include <cstdint>

namespace mm {

// An undirected simple graph (Preliminaries, "Basic Concepts"): n >= 2,
// row_ptr monotone from 0 to nnz (row_ptr: n+1 values, col: nnz), columns in
// range, rows strictly ascending, no self-loops, no isolated vertex (Eq. 2
// divides by rho_u), every edge present in both directions with equal
// weight, node weights c >= 1 and edge weights w >= 1 (NULL = all 1).
bool check_graph(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                 const int32_t* c, const int32_t* w, char* msg, size_t cap);

// A general stress set S ⊇ E in the layout of the k-hop sets (footnote to
// Eq. 1): off[n+1] from 0, non-decreasing, no empty row, fewer than n
// entries per row; hend[u*k + h-1] non-decreasing per row, ending at the
// row length; ids in [0, n), not the row itself, strictly increasing within
// a distance group, no repeat within a row; every pair mirrored at the same
// distance.  nbr holds off[n] ids (may be NULL when off[n] == 0).
bool check_stress_set(int32_t n, int32_t k, const int64_t* off, const int32_t* hend,
                      const int32_t* nbr, char* msg, size_t cap);

// One autotuner record (coarse?, n, entries, k, tile bits, lanes, blocks):
// tile bits 0 (row kernel) or 11..13; lanes a power of two, 8..64 for the
// row kernel, 1..16 or the sliced layout's code 64 when tiled; blocks 0 for
// the row kernel, 0, 2 or 4 when tiled; coarse 0 or 1; n and k in int32
// range, k >= 1; entries >= 0.
bool check_tune_record(const int64_t* rec, int32_t sliced_code);

}  // namespace mm
