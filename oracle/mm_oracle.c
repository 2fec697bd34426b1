/*
 * FP64 CPU oracle for multilevel maxent-stress layout -- implementation.
 * TEST INFRASTRUCTURE ONLY (see mm_oracle.h).  Build: gcc -O2 -fopenmp
 * -ffp-contract=off, no fast-math.
 */
#include "mm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ RNG */

static uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int orc_set_threads(int n) {
    const int prev = omp_get_max_threads();
    if (n >= 1) omp_set_num_threads(n);
    return prev;
}

uint64_t orc_splitmix64_at(uint64_t state, uint64_t i) {
    return sm_mix(state + (i + 1) * 0x9E3779B97F4A7C15ULL);
}

uint64_t orc_stream(uint64_t seed, uint32_t level, uint32_t tag) {
    return seed ^ ((uint64_t)level << 48) ^ ((uint64_t)tag << 32);
}

void orc_draws(uint64_t seed, uint32_t level, uint32_t tag, uint64_t i0,
               int64_t count, uint64_t* out) {
    uint64_t s = orc_stream(seed, level, tag);
    for (int64_t j = 0; j < count; ++j) out[j] = orc_splitmix64_at(s, i0 + (uint64_t)j);
}

static double unit_draw(uint64_t r) { return (double)(r >> 40) * 0x1p-24; }

/* ------------------------------------------------------------- validate */

static int has_edge(const int32_t* rp, const int32_t* col, int32_t u, int32_t v, int64_t* pos) {
    int64_t lo = rp[u], hi = rp[u + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (col[mid] < v) lo = mid + 1; else hi = mid;
    }
    if (lo < rp[u + 1] && col[lo] == v) { if (pos) *pos = lo; return 1; }
    return 0;
}

int orc_validate(int32_t n, const int32_t* rp, const int32_t* col,
                 const int32_t* c, const int32_t* w) {
    if (n < 2) return 1;
    if (rp[0] != 0) return 2;
    for (int32_t u = 0; u < n; ++u)
        if (rp[u + 1] < rp[u]) return 2;
    for (int32_t u = 0; u < n; ++u) {
        if (rp[u + 1] == rp[u]) return 7;
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
            int32_t v = col[e];
            if (v < 0 || v >= n) return 3;
            if (v == u) return 4;
            if (e > rp[u] && col[e - 1] >= v) return 5;
        }
    }
    for (int32_t u = 0; u < n; ++u) {
        if (c && c[u] < 1) return 8;
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
            int64_t back;
            if (!has_edge(rp, col, col[e], u, &back)) return 6;
            if (w) {
                if (w[e] < 1) return 8;
                if (w[back] != w[e]) return 6;
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------- k-hop sets */

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* BFS from u to depth k.  dist[] is -1 everywhere on entry and on exit.
 * list receives S(u) sorted by (hop, v); hcnt[h-1] = entries with hop <= h.
 * Returns |S(u)|. */
static int64_t khop_row(const int32_t* rp, const int32_t* col, int32_t k, int32_t u,
                        int32_t* dist, int32_t* list, int32_t* hcnt) {
    int64_t len = 0;
    dist[u] = 0;
    /* list[0..len) holds visited vertices except u in BFS order */
    /* frontier of hop h-1: for h=1 it is {u} */
    int64_t fr_lo = -1, fr_hi = -1; /* -1 marks the source frontier */
    for (int32_t h = 1; h <= k; ++h) {
        int64_t start = len;
        if (fr_lo < 0) {
            for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
                int32_t v = col[e];
                if (dist[v] < 0) { dist[v] = h; list[len++] = v; }
            }
        } else {
            for (int64_t i = fr_lo; i < fr_hi; ++i) {
                int32_t w = list[i];
                for (int64_t e = rp[w]; e < rp[w + 1]; ++e) {
                    int32_t v = col[e];
                    if (dist[v] < 0) { dist[v] = h; list[len++] = v; }
                }
            }
        }
        qsort(list + start, (size_t)(len - start), sizeof(int32_t), cmp_i32);
        if (hcnt) hcnt[h - 1] = (int32_t)len;
        fr_lo = start; fr_hi = len;
    }
    dist[u] = -1;
    for (int64_t i = 0; i < len; ++i) dist[list[i]] = -1;
    return len;
}

int orc_khop_build(int32_t n, const int32_t* rp, const int32_t* col, int32_t k,
                   int64_t* off, int32_t* hend, int32_t* nbr) {
    if (k < 1) return -1;
    int fail = 0;
    if (nbr == NULL) {
        off[0] = 0;
        int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
        if (!cnt) return -1;
#pragma omp parallel
        {
            int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
            int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
            if (!dist || !list) {
#pragma omp atomic write
                fail = 1;
            } else {
                for (int32_t i = 0; i < n; ++i) dist[i] = -1;
#pragma omp for schedule(dynamic, 64)
                for (int32_t u = 0; u < n; ++u) cnt[u] = khop_row(rp, col, k, u, dist, list, NULL);
            }
            free(dist); free(list);
        }
        for (int32_t u = 0; u < n; ++u) off[u + 1] = off[u] + cnt[u];
        free(cnt);
        return fail ? -1 : 0;
    }
#pragma omp parallel
    {
        int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        if (!dist || !list) {
#pragma omp atomic write
            fail = 1;
        } else {
            for (int32_t i = 0; i < n; ++i) dist[i] = -1;
#pragma omp for schedule(dynamic, 64)
            for (int32_t u = 0; u < n; ++u) {
                int64_t len = khop_row(rp, col, k, u, dist, list, hend ? hend + (int64_t)u * k : NULL);
                memcpy(nbr + off[u], list, sizeof(int32_t) * (size_t)len);
            }
        }
        free(dist); free(list);
    }
    return fail ? -1 : 0;
}

/* ------------------------------------------------------------ r-values */

/* r_q(a, b) = (a - b) / |a - b|^(q+2); (0,0) for coincident points. */
static int rq(double dx, double dy, double q, double* rx, double* ry) {
    double d2 = dx * dx + dy * dy;
    if (d2 == 0.0) { *rx = 0.0; *ry = 0.0; return 0; }
    double f = (q == 0.0) ? 1.0 / d2 : pow(d2, -0.5 * (q + 2.0));
    *rx = dx * f;
    *ry = dy * f;
    return 1;
}

void orc_farfield_exact(int32_t n, const double* xy, double q, double* F) {
#pragma omp parallel for schedule(static)
    for (int32_t u = 0; u < n; ++u) {
        double fx = 0.0, fy = 0.0;
        for (int32_t v = 0; v < n; ++v) {
            if (v == u) continue;
            double rx, ry;
            rq(xy[2 * u] - xy[2 * v], xy[2 * u + 1] - xy[2 * v + 1], q, &rx, &ry);
            fx += rx; fy += ry;
        }
        F[2 * u] = fx; F[2 * u + 1] = fy;
    }
}

/* ------------------------------------------------ cluster far field (Eq. 3)
 * The first two sums of Eq. 3 for every u of one level, in the reading that
 * Section 3.2 gives for an approximation level h > 1 beneath:
 *   sum over v != u with cl1[v] == cl1[u] of r_q(u, v)          (exact, own
 *       cluster of the next coarser level)
 * + sum over coarse vertices j != clh[u] of nu_j r_q(x_u, xp_j)  (level used
 *       for approximation),
 * where nu_j = #{v : clh[v] == j} and xp_j is the c-weighted midpoint of
 * those v.  Vertices whose clh equals clh[u] but whose cl1 differs from
 * cl1[u] contribute nothing (the merged-vertex error of Section 3.2).  With
 * cl1 = clh = identity this is the exact all-pairs sum. */
int orc_cluster_far(int32_t n, const double* xy, const int32_t* c, const int32_t* cl1,
                    int32_t n1, const int32_t* clh, int32_t nh, double q, double* F) {
    for (int32_t v = 0; v < n; ++v)
        if (cl1[v] < 0 || cl1[v] >= n1 || clh[v] < 0 || clh[v] >= nh) return -1;
    double* mid = (double*)calloc(3 * (size_t)(nh > 0 ? nh : 1), sizeof(double));
    int64_t* nu = (int64_t*)calloc((size_t)(nh > 0 ? nh : 1), sizeof(int64_t));
    int64_t* start = (int64_t*)calloc((size_t)n1 + 1, sizeof(int64_t));
    int32_t* memb = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!mid || !nu || !start || !memb) { free(mid); free(nu); free(start); free(memb); return -2; }
    /* weighted midpoints, in ascending v */
    for (int32_t v = 0; v < n; ++v) {
        const double w = c ? (double)c[v] : 1.0;
        const int32_t j = clh[v];
        mid[3 * j] += w * xy[2 * v];
        mid[3 * j + 1] += w * xy[2 * v + 1];
        mid[3 * j + 2] += w;
        nu[j]++;
    }
    for (int32_t j = 0; j < nh; ++j)
        if (nu[j] > 0) { mid[3 * j] /= mid[3 * j + 2]; mid[3 * j + 1] /= mid[3 * j + 2]; }
    /* members of each next-level cluster, ascending */
    for (int32_t v = 0; v < n; ++v) start[cl1[v] + 1]++;
    for (int32_t j = 0; j < n1; ++j) start[j + 1] += start[j];
    {
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n1 + 1));
        if (!fill) { free(mid); free(nu); free(start); free(memb); return -2; }
        memcpy(fill, start, sizeof(int64_t) * ((size_t)n1 + 1));
        for (int32_t v = 0; v < n; ++v) memb[fill[cl1[v]]++] = v;
        free(fill);
    }
#pragma omp parallel for schedule(static)
    for (int32_t u = 0; u < n; ++u) {
        double fx = 0.0, fy = 0.0, rx, ry;
        const int32_t a = cl1[u];
        for (int64_t i = start[a]; i < start[a + 1]; ++i) {
            const int32_t v = memb[i];
            if (v == u) continue;
            rq(xy[2 * u] - xy[2 * v], xy[2 * u + 1] - xy[2 * v + 1], q, &rx, &ry);
            fx += rx; fy += ry;
        }
        for (int32_t j = 0; j < nh; ++j) {
            if (j == clh[u] || nu[j] == 0) continue;
            rq(xy[2 * u] - mid[3 * j], xy[2 * u + 1] - mid[3 * j + 1], q, &rx, &ry);
            fx += (double)nu[j] * rx;
            fy += (double)nu[j] * ry;
        }
        F[2 * u] = fx; F[2 * u + 1] = fy;
    }
    free(mid); free(nu); free(start); free(memb);
    return 0;
}

/* ------------------------------------------------------------ Barnes-Hut */

typedef struct {
    int32_t depth;      /* 0 = root box; 24 = finest cell (leaves report 24) */
    int32_t leaf;
    int64_t first;      /* index into the sorted point order */
    int64_t count;
    uint32_t ox, oy;    /* integer origin of the cell (low 24-depth bits clear) */
    double cx, cy;      /* centre of mass, FP64 */
    double mxx, myy, mxy; /* central second moments per unit mass */
    int32_t child[4];   /* node ids, -1 if empty (internal nodes only) */
    uint64_t prefix;    /* code >> 2*(24-depth) */
} bh_node;

typedef struct {
    bh_node* nodes;
    int64_t count, cap;
    int failed;
} bh_tree;

static int64_t bh_push(bh_tree* t) {
    if (t->count == t->cap) {
        int64_t nc = t->cap ? t->cap * 2 : 1024;
        bh_node* nn = (bh_node*)realloc(t->nodes, sizeof(bh_node) * (size_t)nc);
        if (!nn) { t->failed = 1; return -1; }
        t->nodes = nn; t->cap = nc;
    }
    return t->count++;
}

static uint64_t interleave24(uint32_t ix, uint32_t iy) {
    uint64_t code = 0;
    for (int b = 0; b < 24; ++b) {
        code |= (uint64_t)((ix >> b) & 1u) << (2 * b);
        code |= (uint64_t)((iy >> b) & 1u) << (2 * b + 1);
    }
    return code;
}

/* Build the node covering pts[0..cnt) (point ids in ascending (code, id)
 * order, all inside the cell of depth `depth` with origin (ox, oy)).
 * Child digit at depth t: bit (23-t) of ix gives bit 0, of iy bit 1. */
static int64_t bh_build(bh_tree* t, const int32_t* pts, int64_t first, int64_t cnt,
                        const uint32_t* ix, const uint32_t* iy, const double* xy,
                        int32_t depth, uint32_t ox, uint32_t oy) {
    for (;;) {
        if (cnt == 1 || depth == 24) break;
        int sh = 23 - depth;
        int64_t sub[4] = {0, 0, 0, 0};
        for (int64_t i = 0; i < cnt; ++i) {
            int32_t p = pts[first + i];
            int d = (int)((ix[p] >> sh) & 1u) | (int)(((iy[p] >> sh) & 1u) << 1);
            sub[d]++;
        }
        int nonempty = 0, only = -1;
        for (int d = 0; d < 4; ++d) if (sub[d]) { nonempty++; only = d; }
        if (nonempty > 1) break;
        /* all points in one child: that child is the same node (tight cell) */
        ox |= (uint32_t)(only & 1) << sh;
        oy |= (uint32_t)(only >> 1) << sh;
        depth++;
    }
    if (cnt == 1) { /* a single point: its own finest cell */
        ox = ix[pts[first]];
        oy = iy[pts[first]];
    }
    int64_t id = bh_push(t);
    if (id < 0) return -1;
    bh_node* nd = &t->nodes[id];
    nd->first = first; nd->count = cnt; nd->ox = ox; nd->oy = oy;
    nd->depth = (cnt == 1) ? 24 : depth;
    nd->leaf = (cnt == 1 || depth == 24);
    nd->prefix = interleave24(ox, oy) >> (2 * (24 - nd->depth));
    for (int d = 0; d < 4; ++d) nd->child[d] = -1;
    double sx = 0.0, sy = 0.0;
    for (int64_t i = 0; i < cnt; ++i) {
        int32_t p = pts[first + i];
        sx += xy[2 * p]; sy += xy[2 * p + 1];
    }
    nd->cx = sx / (double)cnt; nd->cy = sy / (double)cnt;
    double sxx = 0.0, syy = 0.0, sxy = 0.0;
    for (int64_t i = 0; i < cnt; ++i) {
        int32_t p = pts[first + i];
        double dx = xy[2 * p] - nd->cx, dy = xy[2 * p + 1] - nd->cy;
        sxx += dx * dx; syy += dy * dy; sxy += dx * dy;
    }
    nd->mxx = sxx / (double)cnt; nd->myy = syy / (double)cnt; nd->mxy = sxy / (double)cnt;
    if (nd->leaf) return id;
    int sh = 23 - depth;
    int64_t pos = first;
    for (int d = 0; d < 4; ++d) {
        /* points are in code order, so each child is a contiguous run */
        int64_t c0 = pos;
        while (pos < first + cnt) {
            int32_t p = pts[pos];
            int dd = (int)((ix[p] >> sh) & 1u) | (int)(((iy[p] >> sh) & 1u) << 1);
            if (dd != d) break;
            pos++;
        }
        if (pos > c0) {
            uint32_t cox = ox | ((uint32_t)(d & 1) << sh);
            uint32_t coy = oy | ((uint32_t)(d >> 1) << sh);
            int64_t ch = bh_build(t, pts, c0, pos - c0, ix, iy, xy, depth + 1, cox, coy);
            if (ch < 0) return -1;
            t->nodes[id].child[d] = (int32_t)ch;
        }
    }
    return id;
}

typedef struct {
    const bh_tree* t;
    const int32_t* pts;
    const uint32_t *ix, *iy;
    const double* xy;
    double q, theta2;
    double xmin, ymin, scale; /* box origin and quanta per unit length */
} bh_ctx;

static void bh_visit(const bh_ctx* c, int64_t id, int32_t u, double* fx, double* fy,
                     int64_t* acc, int64_t* pairs, int64_t* coinc) {
    const bh_node* nd = &c->t->nodes[id];
    double xu = c->xy[2 * u], yu = c->xy[2 * u + 1];
    if (nd->leaf) {
        for (int64_t i = 0; i < nd->count; ++i) {
            int32_t v = c->pts[nd->first + i];
            if (v == u) continue;
            double rx, ry;
            if (rq(xu - c->xy[2 * v], yu - c->xy[2 * v + 1], c->q, &rx, &ry)) {
                *fx += rx; *fy += ry; (*pairs)++;
            } else {
                (*coinc)++;
            }
        }
        return;
    }
    int sh = 24 - nd->depth;
    int contains = ((c->ix[u] >> sh) == (nd->ox >> sh)) && ((c->iy[u] >> sh) == (nd->oy >> sh));
    if (!contains) {
        int64_t S = (int64_t)1 << sh;
        int64_t dx = 2 * (int64_t)c->ix[u] + 1 - (2 * (int64_t)nd->ox + S);
        int64_t dy = 2 * (int64_t)c->iy[u] + 1 - (2 * (int64_t)nd->oy + S);
        double d4 = (double)(dx * dx + dy * dy);
        double s4 = (double)(4 * S * S);
        if (c->theta2 * d4 > s4) {
            double rx, ry;
            if (rq(xu - nd->cx, yu - nd->cy, c->q, &rx, &ry)) {
                *fx += (double)nd->count * rx; *fy += (double)nd->count * ry;
            } else {
                (*coinc)++;
            }
            (*acc)++;
            return;
        }
    }
    for (int d = 0; d < 4; ++d)
        if (nd->child[d] >= 0) bh_visit(c, nd->child[d], u, fx, fy, acc, pairs, coinc);
}

static void bh_preorder(const bh_tree* t, int64_t id, int64_t* out, int64_t cap, int64_t* k) {
    const bh_node* nd = &t->nodes[id];
    if (*k < cap) {
        int64_t* o = out + 5 * (*k);
        o[0] = nd->depth; o[1] = nd->first; o[2] = nd->count; o[3] = nd->leaf;
        o[4] = (int64_t)nd->prefix;
    }
    (*k)++;
    if (nd->leaf) return;
    for (int d = 0; d < 4; ++d)
        if (nd->child[d] >= 0) bh_preorder(t, nd->child[d], out, cap, k);
}

typedef struct { uint64_t code; int32_t id; } code_id;
static int cmp_code_id(const void* a, const void* b) {
    const code_id* x = (const code_id*)a; const code_id* y = (const code_id*)b;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

typedef struct {
    bh_tree t;
    int64_t root;
    uint32_t *ix, *iy;
    int32_t* pts;
    double xmin, ymin, scale;
} bh_setup;

static void bh_setup_free(bh_setup* b) {
    free(b->t.nodes); free(b->ix); free(b->iy); free(b->pts);
}

/* Box, quantisation, (code, id) order and the quadtree of xy. */
static int bh_setup_build(int32_t n, const double* xy, uint64_t* codes_out, int32_t* order_out,
                          bh_setup* b) {
    memset(b, 0, sizeof(*b));
    double xmin = xy[0], xmax = xy[0], ymin = xy[1], ymax = xy[1];
    for (int32_t v = 1; v < n; ++v) {
        if (xy[2 * v] < xmin) xmin = xy[2 * v];
        if (xy[2 * v] > xmax) xmax = xy[2 * v];
        if (xy[2 * v + 1] < ymin) ymin = xy[2 * v + 1];
        if (xy[2 * v + 1] > ymax) ymax = xy[2 * v + 1];
    }
    double ext = fmax(xmax - xmin, ymax - ymin);
    int e = 0;
    if (ext > 0.0) {
        int ex;
        double m = frexp(ext, &ex); /* ext = m 2^ex, m in [0.5, 1) */
        e = (m == 0.5) ? ex - 1 : ex;
    }
    double scale = ldexp(1.0, 24 - e);
    b->xmin = xmin; b->ymin = ymin; b->scale = scale;
    b->ix = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    b->iy = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    b->pts = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    code_id* ci = (code_id*)malloc(sizeof(code_id) * (size_t)n);
    if (!b->ix || !b->iy || !ci || !b->pts) { free(ci); bh_setup_free(b); return -1; }
    for (int32_t v = 0; v < n; ++v) {
        double fxq = floor((xy[2 * v] - xmin) * scale);
        double fyq = floor((xy[2 * v + 1] - ymin) * scale);
        if (fxq > 16777215.0) fxq = 16777215.0;
        if (fyq > 16777215.0) fyq = 16777215.0;
        if (fxq < 0.0) fxq = 0.0;
        if (fyq < 0.0) fyq = 0.0;
        b->ix[v] = (uint32_t)fxq; b->iy[v] = (uint32_t)fyq;
        ci[v].code = interleave24(b->ix[v], b->iy[v]);
        ci[v].id = v;
        if (codes_out) codes_out[v] = ci[v].code;
    }
    qsort(ci, (size_t)n, sizeof(code_id), cmp_code_id);
    for (int32_t i = 0; i < n; ++i) b->pts[i] = ci[i].id;
    if (order_out) memcpy(order_out, b->pts, sizeof(int32_t) * (size_t)n);
    free(ci);
    b->root = bh_build(&b->t, b->pts, 0, n, b->ix, b->iy, xy, 0, 0u, 0u);
    if (b->root < 0 || b->t.failed) { bh_setup_free(b); return -1; }
    return 0;
}

int orc_bh(int32_t n, const double* xy, double q, double theta, double* F,
           uint64_t* codes_out, int32_t* order_out, int64_t* nodes_out, int64_t node_cap,
           int64_t* stats) {
    bh_setup b;
    if (bh_setup_build(n, xy, codes_out, order_out, &b) != 0) return -1;
    bh_ctx c = {&b.t, b.pts, b.ix, b.iy, xy, q, theta * theta, b.xmin, b.ymin, b.scale};
    int64_t acc = 0, pairs = 0, coinc = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : acc, pairs, coinc)
    for (int32_t u = 0; u < n; ++u) {
        double fx = 0.0, fy = 0.0;
        bh_visit(&c, b.root, u, &fx, &fy, &acc, &pairs, &coinc);
        F[2 * u] = fx; F[2 * u + 1] = fy;
    }
    if (nodes_out) {
        int64_t k = 0;
        bh_preorder(&b.t, b.root, nodes_out, node_cap, &k);
    }
    if (stats) { stats[0] = acc; stats[1] = pairs; stats[2] = coinc; stats[3] = b.t.count; }
    bh_setup_free(&b);
    return 0;
}

/* ------------------------------------------------ learned far field (q = 0)
 * A cell C accepted for target u contributes m r(x_u - com) plus a learned
 * correction kappa (h0 e + h1 p): e = (x_u - com)/d, p = e rotated by +90
 * degrees, kappa = m t^2 / d with t = s/d, s the side of C's tight cell,
 * and h = MLP(features).  The scaling makes h the cell's dimensionless
 * multipole coefficient: for a far target h tends to
 * (mu_ee - mu_pp, -2 mu_ep), the quadrupole term of the expansion of
 * sum_v 1/conj(z - w_v). */

#define MLP_IN 8
#define MLP_H 64
#define MLP_OUT 2

/* Features of (u, C): t, centroid offset from the cell centre along e and p
 * (in units of s), second central moments per unit mass rotated into the
 * (e, p) frame (units of s^2), log2(m)/16, and a zero pad.  *ke receives
 * kappa e (kappa p is its rotation).  Returns 0 when x_u == com. */
static int cell_features(const bh_ctx* c, const bh_node* nd, double xu, double yu, double* f,
                         double* kex, double* key) {
    double dx = xu - nd->cx, dy = yu - nd->cy;
    double d2 = dx * dx + dy * dy;
    if (d2 == 0.0) return 0;
    double d = sqrt(d2);
    double ex = dx / d, ey = dy / d, px = -ey, py = ex;
    double S = ldexp(1.0, 24 - nd->depth);
    double s = S / c->scale;
    double gx = c->xmin + ((double)nd->ox + 0.5 * S) / c->scale;
    double gy = c->ymin + ((double)nd->oy + 0.5 * S) / c->scale;
    double ox = nd->cx - gx, oy = nd->cy - gy;
    double s2 = s * s;
    double t = s / d;
    f[0] = t;
    f[1] = (ox * ex + oy * ey) / s;
    f[2] = (ox * px + oy * py) / s;
    f[3] = (ex * ex * nd->mxx + 2.0 * ex * ey * nd->mxy + ey * ey * nd->myy) / s2;
    f[4] = (px * px * nd->mxx + 2.0 * px * py * nd->mxy + py * py * nd->myy) / s2;
    f[5] = (ex * px * nd->mxx + (ex * py + ey * px) * nd->mxy + ey * py * nd->myy) / s2;
    f[6] = log2((double)nd->count) / 16.0;
    f[7] = 0.0;
    double kappa = (double)nd->count * t * t / d;
    *kex = kappa * ex;
    *key = kappa * ey;
    return 1;
}

/* Weights: W1[64][8], b1[64], W2[64][64], b2[64], W3[2][64], b3[2]. */
static void mlp_forward(const double* w, const double* f, double* h) {
    const double* W1 = w;
    const double* b1 = W1 + MLP_H * MLP_IN;
    const double* W2 = b1 + MLP_H;
    const double* b2 = W2 + MLP_H * MLP_H;
    const double* W3 = b2 + MLP_H;
    const double* b3 = W3 + MLP_OUT * MLP_H;
    double a1[MLP_H], a2[MLP_H];
    for (int o = 0; o < MLP_H; ++o) {
        double z = b1[o];
        for (int i = 0; i < MLP_IN; ++i) z += W1[o * MLP_IN + i] * f[i];
        a1[o] = z > 0.0 ? z : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) {
        double z = b2[o];
        for (int i = 0; i < MLP_H; ++i) z += W2[o * MLP_H + i] * a1[i];
        a2[o] = z > 0.0 ? z : 0.0;
    }
    for (int o = 0; o < MLP_OUT; ++o) {
        double z = b3[o];
        for (int i = 0; i < MLP_H; ++i) z += W3[o * MLP_H + i] * a2[i];
        h[o] = z;
    }
}

typedef struct {
    int64_t cap, count;
    int32_t* u;
    int64_t* node;
    double *feat, *target, *coef;
} sample_sink;

/* Depth-first visit as bh_visit (q = 0).  Leaves add exact terms; an accepted
 * cell adds its plain term and, when `w` is given, the learned correction,
 * or, when `sk` is given, is recorded as a training sample: features,
 * kappa e, and the exact residual of the cell in h units. */
static void bh_visit_learned(const bh_ctx* c, int64_t id, int32_t u, const double* w,
                             sample_sink* sk, double* fx, double* fy) {
    const bh_node* nd = &c->t->nodes[id];
    double xu = c->xy[2 * u], yu = c->xy[2 * u + 1];
    if (nd->leaf) {
        for (int64_t i = 0; i < nd->count; ++i) {
            int32_t v = c->pts[nd->first + i];
            if (v == u) continue;
            double rx, ry;
            if (rq(xu - c->xy[2 * v], yu - c->xy[2 * v + 1], 0.0, &rx, &ry)) {
                *fx += rx; *fy += ry;
            }
        }
        return;
    }
    int sh = 24 - nd->depth;
    int contains = ((c->ix[u] >> sh) == (nd->ox >> sh)) && ((c->iy[u] >> sh) == (nd->oy >> sh));
    if (!contains) {
        int64_t S = (int64_t)1 << sh;
        int64_t dx = 2 * (int64_t)c->ix[u] + 1 - (2 * (int64_t)nd->ox + S);
        int64_t dy = 2 * (int64_t)c->iy[u] + 1 - (2 * (int64_t)nd->oy + S);
        double d4 = (double)(dx * dx + dy * dy);
        double s4 = (double)(4 * S * S);
        if (c->theta2 * d4 > s4) {
            double rx, ry;
            double m = (double)nd->count;
            if (rq(xu - nd->cx, yu - nd->cy, 0.0, &rx, &ry)) {
                *fx += m * rx; *fy += m * ry;
            }
            double f[MLP_IN], kex, key;
            if (cell_features(c, nd, xu, yu, f, &kex, &key)) {
                if (w) {
                    double h[MLP_OUT];
                    mlp_forward(w, f, h);
                    /* kappa (h0 e + h1 p), p = (-e_y, e_x) */
                    *fx += h[0] * kex - h[1] * key;
                    *fy += h[0] * key + h[1] * kex;
                }
                if (sk && sk->count < sk->cap) {
                    int64_t j = sk->count;
                    double ex0 = 0.0, ey0 = 0.0;
                    for (int64_t i = 0; i < nd->count; ++i) {
                        int32_t v = c->pts[nd->first + i];
                        double ax, ay;
                        if (rq(xu - c->xy[2 * v], yu - c->xy[2 * v + 1], 0.0, &ax, &ay)) {
                            ex0 += ax; ey0 += ay;
                        }
                    }
                    double Rx = ex0 - m * rx, Ry = ey0 - m * ry;
                    double k2 = kex * kex + key * key; /* kappa^2 */
                    sk->u[j] = u;
                    sk->node[j] = id;
                    for (int i = 0; i < MLP_IN; ++i) sk->feat[MLP_IN * j + i] = f[i];
                    /* h* = (R.e, R.p) / kappa = (R.(kappa e), R.(kappa p)) / kappa^2 */
                    sk->target[2 * j] = (Rx * kex + Ry * key) / k2;
                    sk->target[2 * j + 1] = (-Rx * key + Ry * kex) / k2;
                    sk->coef[2 * j] = kex;
                    sk->coef[2 * j + 1] = key;
                }
                if (sk) sk->count++;
            }
            return;
        }
    }
    for (int d = 0; d < 4; ++d)
        if (nd->child[d] >= 0) bh_visit_learned(c, nd->child[d], u, w, sk, fx, fy);
}

int orc_far_samples(int32_t n, const double* xy, double theta, int64_t cap, int32_t* u_out,
                    int64_t* node_out, double* feat_out, double* target_out, double* coef_out,
                    int64_t* count) {
    bh_setup b;
    if (bh_setup_build(n, xy, NULL, NULL, &b) != 0) return -1;
    bh_ctx c = {&b.t, b.pts, b.ix, b.iy, xy, 0.0, theta * theta, b.xmin, b.ymin, b.scale};
    sample_sink sk = {cap, 0, u_out, node_out, feat_out, target_out, coef_out};
    /* sequential: samples are recorded in (u, visit) order */
    for (int32_t u = 0; u < n; ++u) {
        double fx = 0.0, fy = 0.0;
        bh_visit_learned(&c, b.root, u, NULL, &sk, &fx, &fy);
    }
    *count = sk.count;
    bh_setup_free(&b);
    return 0;
}

int orc_bh_learned(int32_t n, const double* xy, double theta, const double* weights,
                   double* F) {
    bh_setup b;
    if (bh_setup_build(n, xy, NULL, NULL, &b) != 0) return -1;
    bh_ctx c = {&b.t, b.pts, b.ix, b.iy, xy, 0.0, theta * theta, b.xmin, b.ymin, b.scale};
#pragma omp parallel for schedule(dynamic, 256)
    for (int32_t u = 0; u < n; ++u) {
        double fx = 0.0, fy = 0.0;
        bh_visit_learned(&c, b.root, u, weights, NULL, &fx, &fy);
        F[2 * u] = fx; F[2 * u + 1] = fy;
    }
    bh_setup_free(&b);
    return 0;
}

int orc_bh_learned_rows(int32_t n, const double* xy, double theta, const double* weights,
                        const int32_t* rows, int32_t nrows, double* F) {
    bh_setup b;
    if (bh_setup_build(n, xy, NULL, NULL, &b) != 0) return -1;
    bh_ctx c = {&b.t, b.pts, b.ix, b.iy, xy, 0.0, theta * theta, b.xmin, b.ymin, b.scale};
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t i = 0; i < nrows; ++i) {
        double fx = 0.0, fy = 0.0;
        bh_visit_learned(&c, b.root, rows[i], weights, NULL, &fx, &fy);
        F[2 * i] = fx; F[2 * i + 1] = fy;
    }
    bh_setup_free(&b);
    return 0;
}

void orc_mlp_forward(const double* weights, int64_t count, const double* feat, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < count; ++j) mlp_forward(weights, feat + MLP_IN * j, out + 2 * j);
}

/* --------------------------------------------------------------- sweep */

static double target_dist(int32_t hop, int32_t level, const int32_t* c, int32_t u, int32_t v,
                          double scale) {
    if (level == 0) return (double)hop;
    double cu = c ? (double)c[u] : 1.0, cv = c ? (double)c[v] : 1.0;
    return (double)hop * (sqrt(cu) + sqrt(cv)) * scale;
}

/* Stress terms of Eq. 2 over the list S(u) (ids `lst`, cumulative hop
 * counts `hc`): A, C (sum of r over S) and rho. */
static void stress_terms(int32_t u, int32_t level, int32_t k, const int32_t* lst,
                         const int32_t* hc, const int32_t* c, double scale, const double* x,
                         double q, double* A, double* C, double* rho) {
    double ax = 0.0, ay = 0.0, cx = 0.0, cy = 0.0, r = 0.0;
    int32_t e = 0;
    for (int32_t h = 1; h <= k; ++h) {
        for (; e < hc[h - 1]; ++e) {
            int32_t v = lst[e];
            double d = target_dist(h, level, c, u, v, scale);
            double w = 1.0 / (d * d);
            double dx = x[2 * u] - x[2 * v], dy = x[2 * u + 1] - x[2 * v + 1];
            double D = sqrt(dx * dx + dy * dy);
            r += w;
            if (D == 0.0) {
                ax += w * x[2 * v]; ay += w * x[2 * v + 1];
                continue;
            }
            ax += w * (x[2 * v] + d * dx / D);
            ay += w * (x[2 * v + 1] + d * dy / D);
            double rx, ry;
            rq(dx, dy, q, &rx, &ry);
            cx += rx; cy += ry;
        }
    }
    A[0] = ax; A[1] = ay; C[0] = cx; C[1] = cy; *rho = r;
}

static void delta_sums(int32_t n, const double* x, const double* xo, double* delta) {
    double num = 0.0, den = 0.0;
    for (int32_t u = 0; u < n; ++u) {
        double dx = xo[2 * u] - x[2 * u], dy = xo[2 * u + 1] - x[2 * u + 1];
        num += dx * dx + dy * dy;
        den += x[2 * u] * x[2 * u] + x[2 * u + 1] * x[2 * u + 1];
    }
    delta[0] = num; delta[1] = den;
}

int orc_sweep(int32_t n, int32_t level, int32_t k, const int64_t* off, const int32_t* hend,
              const int32_t* nbr, const int32_t* c, double scale, const double* x,
              const double* F, double alpha, double q, double* xout, double* delta) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int32_t u = 0; u < n; ++u) {
        double A[2], C[2], rho;
        stress_terms(u, level, k, nbr + off[u], hend + (int64_t)u * k, c, scale, x, q, A, C, &rho);
        xout[2 * u] = (A[0] + alpha * (F[2 * u] - C[0])) / rho;
        xout[2 * u + 1] = (A[1] + alpha * (F[2 * u + 1] - C[1])) / rho;
    }
    if (delta) delta_sums(n, x, xout, delta);
    return 0;
}

int orc_sweep_direct(int32_t n, int32_t level, int32_t k, const int64_t* off,
                     const int32_t* hend, const int32_t* nbr, const int32_t* c, double scale,
                     const double* x, double alpha, double q, double* xout, double* delta) {
    int fail = 0;
#pragma omp parallel
    {
        char* inS = (char*)calloc((size_t)n, 1);
        if (!inS) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int32_t u = 0; u < n; ++u) {
                double A[2], C[2], rho;
                const int32_t* lst = nbr + off[u];
                int64_t len = off[u + 1] - off[u];
                stress_terms(u, level, k, lst, hend + (int64_t)u * k, c, scale, x, q, A, C, &rho);
                for (int64_t i = 0; i < len; ++i) inS[lst[i]] = 1;
                double ex = 0.0, ey = 0.0;
                for (int32_t v = 0; v < n; ++v) {
                    if (v == u || inS[v]) continue;
                    double rx, ry;
                    rq(x[2 * u] - x[2 * v], x[2 * u + 1] - x[2 * v + 1], q, &rx, &ry);
                    ex += rx; ey += ry;
                }
                for (int64_t i = 0; i < len; ++i) inS[lst[i]] = 0;
                xout[2 * u] = (A[0] + alpha * ex) / rho;
                xout[2 * u + 1] = (A[1] + alpha * ey) / rho;
            }
        }
        free(inS);
    }
    if (fail) return -1;
    if (delta) delta_sums(n, x, xout, delta);
    return 0;
}

int orc_sweep_rows(int32_t n, const int32_t* rp, const int32_t* col, int32_t level, int32_t k,
                   const int32_t* c, double scale, const double* x, const double* F,
                   double alpha, double q, const int32_t* rows, int32_t nrows,
                   double* xout_rows, int64_t* set_sizes) {
    int fail = 0;
#pragma omp parallel
    {
        int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        int32_t* hc = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
        if (!dist || !list || !hc) {
#pragma omp atomic write
            fail = 1;
        } else {
            for (int32_t i = 0; i < n; ++i) dist[i] = -1;
#pragma omp for schedule(dynamic, 1)
            for (int32_t i = 0; i < nrows; ++i) {
                int32_t u = rows[i];
                int64_t len = khop_row(rp, col, k, u, dist, list, hc);
                if (set_sizes) set_sizes[i] = len;
                double A[2], C[2], rho;
                stress_terms(u, level, k, list, hc, c, scale, x, q, A, C, &rho);
                xout_rows[2 * i] = (A[0] + alpha * (F[2 * u] - C[0])) / rho;
                xout_rows[2 * i + 1] = (A[1] + alpha * (F[2 * u + 1] - C[1])) / rho;
            }
        }
        free(dist); free(list); free(hc);
    }
    return fail ? -1 : 0;
}

/* ------------------------------------------------------ label propagation */

int orc_lp(int32_t n, const int32_t* rp, const int32_t* col, const int32_t* c,
           const int32_t* w, double U, int32_t rounds, uint64_t seed, int32_t level_h,
           int32_t* label, int32_t* moves) {
    int64_t* W = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int32_t* prop = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);   /* proposed label or -1 */
    int64_t* used = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);   /* admission prefix sums */
    int32_t* active = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!W || !prop || !used || !active) { free(W); free(prop); free(used); free(active); return -1; }
    int r_done = 0;
    for (int32_t r = 0; r < rounds; ++r) {
        uint64_t st = orc_stream(seed, (uint32_t)level_h, 16u + (uint32_t)r);
        for (int32_t v = 0; v < n; ++v) active[v] = (int32_t)(orc_splitmix64_at(st, (uint64_t)v) & 1u);
        int32_t round_moves = 0;
        for (int32_t s = 0; s < 2; ++s) {
            for (int32_t v = 0; v < n; ++v) W[v] = 0;
            for (int32_t v = 0; v < n; ++v) W[label[v]] += c ? c[v] : 1;
            int fail = 0;
#pragma omp parallel
            {
                int64_t* score = (int64_t*)calloc((size_t)n, sizeof(int64_t));
                int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
                if (!score || !touched) {
#pragma omp atomic write
                    fail = 1;
                } else {
#pragma omp for schedule(dynamic, 256)
                    for (int32_t v = 0; v < n; ++v) {
                        prop[v] = -1;
                        if (active[v] != s) continue;
                        int32_t nt = 0;
                        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
                            int32_t L = label[col[e]];
                            if (score[L] == 0) touched[nt++] = L;
                            score[L] += w ? w[e] : 1;
                        }
                        int32_t own = label[v];
                        int32_t best = own;
                        int64_t best_sc = score[own];
                        int64_t cv = c ? c[v] : 1;
                        for (int32_t i = 0; i < nt; ++i) {
                            int32_t L = touched[i];
                            if (L == own) continue;
                            int64_t sc = score[L];
                            if ((double)(W[L] + cv) > U) continue; /* infeasible */
                            if (sc > best_sc || (sc == best_sc && best != own && L < best)) {
                                best = L; best_sc = sc;
                            }
                        }
                        for (int32_t i = 0; i < nt; ++i) score[touched[i]] = 0;
                        if (best != own) prop[v] = best;
                    }
                }
                free(score); free(touched);
            }
            if (fail) { free(W); free(prop); free(used); free(active); return -1; }
            /* admission: per target in ascending v, prefix sums of c */
            for (int32_t L = 0; L < n; ++L) used[L] = W[L];
            int32_t sub_moves = 0;
            for (int32_t v = 0; v < n; ++v) {
                if (prop[v] < 0) continue;
                int32_t L = prop[v];
                used[L] += c ? c[v] : 1;
                if ((double)used[L] <= U) {
                    prop[v] = L;       /* admitted */
                } else {
                    prop[v] = -2 - L;  /* rejected, remembered for clarity */
                }
            }
            for (int32_t v = 0; v < n; ++v) {
                if (prop[v] >= 0) { label[v] = prop[v]; sub_moves++; }
            }
            round_moves += sub_moves;
        }
        if (moves) moves[r] = round_moves;
        r_done = r + 1;
        if (round_moves == 0) break;
    }
    free(W); free(prop); free(used); free(active);
    return r_done;
}

/* ------------------------------------------------------------ contraction */

int32_t orc_contract(int32_t n, const int32_t* rp, const int32_t* col, const int32_t* c,
                     const int32_t* w, const int32_t* label, int32_t* cluster,
                     int32_t* crp, int32_t* ccol, int32_t* cc, int32_t* cw, int64_t* cnnz) {
    /* rank of each distinct label in ascending order */
    char* present = (char*)calloc((size_t)n, 1);
    int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!present || !rank) { free(present); free(rank); return -1; }
    for (int32_t v = 0; v < n; ++v) present[label[v]] = 1;
    int32_t nc = 0;
    for (int32_t L = 0; L < n; ++L) rank[L] = present[L] ? nc++ : -1;
    for (int32_t v = 0; v < n; ++v) cluster[v] = rank[label[v]];
    free(present); free(rank);
    /* members of each coarse vertex, in ascending fine id */
    int32_t* mstart = (int32_t*)calloc((size_t)nc + 1, sizeof(int32_t));
    int32_t* members = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int64_t* acc = (int64_t*)calloc((size_t)nc, sizeof(int64_t));
    int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)nc);
    if (!mstart || !members || !acc || !touched) {
        free(mstart); free(members); free(acc); free(touched); return -1;
    }
    for (int32_t v = 0; v < n; ++v) mstart[cluster[v] + 1]++;
    for (int32_t i = 0; i < nc; ++i) mstart[i + 1] += mstart[i];
    {
        int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)nc);
        for (int32_t i = 0; i < nc; ++i) fill[i] = mstart[i];
        for (int32_t v = 0; v < n; ++v) members[fill[cluster[v]]++] = v;
        free(fill);
    }
    int64_t e_out = 0;
    crp[0] = 0;
    for (int32_t U = 0; U < nc; ++U) {
        int64_t wsum = 0;
        int32_t nt = 0;
        for (int32_t i = mstart[U]; i < mstart[U + 1]; ++i) {
            int32_t v = members[i];
            wsum += c ? c[v] : 1;
            for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
                int32_t V = cluster[col[e]];
                if (V == U) continue;
                if (acc[V] == 0) touched[nt++] = V;
                acc[V] += w ? w[e] : 1;
            }
        }
        cc[U] = (int32_t)wsum;
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        for (int32_t i = 0; i < nt; ++i) {
            ccol[e_out] = touched[i];
            cw[e_out] = (int32_t)acc[touched[i]];
            acc[touched[i]] = 0;
            e_out++;
        }
        crp[U + 1] = (int32_t)e_out;
    }
    *cnnz = e_out;
    free(mstart); free(members); free(acc); free(touched);
    return nc;
}

/* ------------------------------------------------ initial layout, prolong */

void orc_init_layout(int32_t n, uint64_t seed, int32_t level, double* xy) {
    uint64_t st = orc_stream(seed, (uint32_t)level, 1u);
    for (int32_t v = 0; v < n; ++v) {
        xy[2 * v] = unit_draw(orc_splitmix64_at(st, 2 * (uint64_t)v));
        xy[2 * v + 1] = unit_draw(orc_splitmix64_at(st, 2 * (uint64_t)v + 1));
    }
}

void orc_prolong(int32_t n_fine, const int32_t* cluster, const int32_t* coarse_c,
                 const double* coarse_xy, uint64_t seed, int32_t level, double* fine_xy) {
    const double two_pi = 6.283185307179586476925286766559;
    uint64_t st = orc_stream(seed, (uint32_t)level, 2u);
    for (int32_t v = 0; v < n_fine; ++v) {
        int32_t p = cluster[v];
        double phi = two_pi * unit_draw(orc_splitmix64_at(st, 2 * (uint64_t)v));
        double rad = sqrt((double)(coarse_c ? coarse_c[p] : 1)) *
                     unit_draw(orc_splitmix64_at(st, 2 * (uint64_t)v + 1));
        fine_xy[2 * v] = coarse_xy[2 * p] + rad * cos(phi);
        fine_xy[2 * v + 1] = coarse_xy[2 * p + 1] + rad * sin(phi);
    }
}

/* -------------------------------------------------------------- objectives */

int orc_objective(int32_t n, int32_t level, int32_t k, const int64_t* off,
                  const int32_t* hend, const int32_t* nbr, const int32_t* c, double scale,
                  const double* x, double q, double* out) {
    double* st_row = (double*)calloc((size_t)n, sizeof(double));
    double* en_row = (double*)calloc((size_t)n, sizeof(double));
    int64_t* co_row = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    int fail = !st_row || !en_row || !co_row;
    if (!fail) {
#pragma omp parallel
        {
            int32_t* hopof = (int32_t*)calloc((size_t)n, sizeof(int32_t));
            if (!hopof) {
#pragma omp atomic write
                fail = 1;
            } else {
#pragma omp for schedule(dynamic, 64)
                for (int32_t u = 0; u < n; ++u) {
                    const int32_t* lst = nbr + off[u];
                    const int32_t* hc = hend + (int64_t)u * k;
                    int32_t e = 0;
                    for (int32_t h = 1; h <= k; ++h)
                        for (; e < hc[h - 1]; ++e) hopof[lst[e]] = h;
                    double st = 0.0, en = 0.0;
                    int64_t co = 0;
                    for (int32_t v = u + 1; v < n; ++v) {
                        double dx = x[2 * u] - x[2 * v], dy = x[2 * u + 1] - x[2 * v + 1];
                        double D = sqrt(dx * dx + dy * dy);
                        if (hopof[v]) {
                            double d = target_dist(hopof[v], level, c, u, v, scale);
                            st += (D - d) * (D - d) / (d * d);
                        } else if (D == 0.0) {
                            co++;
                        } else {
                            en += (q == 0.0) ? log(D) : -pow(D, -q) / q;
                        }
                    }
                    for (int32_t i = 0; i < e; ++i) hopof[lst[i]] = 0;
                    st_row[u] = st; en_row[u] = en; co_row[u] = co;
                }
            }
            free(hopof);
        }
    }
    if (!fail) {
        double st = 0.0, en = 0.0, co = 0.0;
        for (int32_t u = 0; u < n; ++u) { st += st_row[u]; en += en_row[u]; co += (double)co_row[u]; }
        out[0] = st; out[1] = en; out[2] = co;
    }
    free(st_row); free(en_row); free(co_row);
    return fail ? -1 : 0;
}

int orc_full_stress(int32_t n, const int32_t* rp, const int32_t* col, const double* x,
                    double* out) {
    double* s1 = (double*)calloc((size_t)n, sizeof(double));
    double* s2 = (double*)calloc((size_t)n, sizeof(double));
    double* s0 = (double*)calloc((size_t)n, sizeof(double));
    int fail = !s1 || !s2 || !s0;
    /* pass 1: sum D/d, sum (D/d)^2, and F(x) unscaled */
    for (int pass = 0; pass < 2 && !fail; ++pass) {
        double sstar = 0.0;
        if (pass == 1) {
            double a = 0.0, b = 0.0;
            for (int32_t u = 0; u < n; ++u) { a += s1[u]; b += s2[u]; }
            sstar = (b > 0.0) ? a / b : 1.0;
            out[1] = sstar;
        }
#pragma omp parallel
        {
            int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
            int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
            if (!dist || !queue) {
#pragma omp atomic write
                fail = 1;
            } else {
#pragma omp for schedule(dynamic, 16)
                for (int32_t u = 0; u < n; ++u) {
                    for (int32_t i = 0; i < n; ++i) dist[i] = -1;
                    int64_t head = 0, tail = 0;
                    dist[u] = 0; queue[tail++] = u;
                    while (head < tail) {
                        int32_t a = queue[head++];
                        for (int64_t e = rp[a]; e < rp[a + 1]; ++e) {
                            int32_t b = col[e];
                            if (dist[b] < 0) { dist[b] = dist[a] + 1; queue[tail++] = b; }
                        }
                    }
                    double a1 = 0.0, a2 = 0.0, a0 = 0.0;
                    for (int32_t v = u + 1; v < n; ++v) {
                        if (dist[v] <= 0) continue;
                        double d = (double)dist[v];
                        double dx = x[2 * u] - x[2 * v], dy = x[2 * u + 1] - x[2 * v + 1];
                        double D = sqrt(dx * dx + dy * dy);
                        if (pass == 0) {
                            a1 += D / d; a2 += (D / d) * (D / d);
                            a0 += (D - d) * (D - d) / (d * d);
                        } else {
                            a0 += (sstar * D - d) * (sstar * D - d) / (d * d);
                        }
                    }
                    if (pass == 0) { s1[u] = a1; s2[u] = a2; s0[u] = a0; }
                    else s0[u] = a0;
                }
            }
            free(dist); free(queue);
        }
        if (!fail) {
            double f = 0.0;
            for (int32_t u = 0; u < n; ++u) f += s0[u];
            if (pass == 0) out[0] = f; else out[2] = f;
        }
    }
    free(s1); free(s2); free(s0);
    return fail ? -1 : 0;
}
