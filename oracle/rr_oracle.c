/*
 * rr_oracle.c -- plain CPU reference for the red-rec solver and the batching routine of
 * "Efficient algorithms to solve atom reconfiguration problems III" (arXiv 2504.06182).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test-suite, by the smoke check and
 * by the CPU-baseline leg of the benchmark, and by nothing else.  It shares no code, header,
 * table or helper with the HIP library; the two agree only on the byte layout of arguments.
 *
 * Style: single-threaded loops that follow the paper's steps in its order; quadratic scans
 * where the definition is a scan; no blocking, fusion or reordering.  Where the paper leaves a
 * choice open, the reading taken is stated where it is used.
 *
 * Pins (tests/): exact-1D window against brute-force assignment and the quadratic worst case of
 * §III.A; every solve replayed move by move (source occupied, path free, one token per trap,
 * Manhattan length, target covered iff status OK, feasibility formula); the pair loop against
 * hand-worked fixtures and a naive re-implementation of the pairing rule; batches replayed
 * step by step against the solve's final grid; the indexed batching form equal to the literal
 * one on fixtures and random instances.
 * Parity unpinned: the tie-break conventions (leftmost E1D window, Stage-H centring offset,
 * pair-key tie order, receiver split tie, co-location order, constraint reading) are readings,
 * not results the paper fixes; they are pinned only by the hand-worked fixtures.
 *
 * Geometry: grid W x H, columns x = 0..W-1 left to right, rows y = 0..H-1 bottom to top
 * (§III.C).  Target T = [x0,x1) x [y0,y1).  "Band" rows are [y0,y1), "central" columns
 * [x0,x1); the rest are reservoir rows / side columns.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { O_OK = 0, O_INFEASIBLE = 1, O_E_INVAL = -1, O_E_CAPACITY = -2, O_E_NOMEM = -4, O_E_INTERNAL = -5 };
enum { O_LAMBDA_LINE_OR_COL = 0, O_LAMBDA_ALONG = 1, O_LAMBDA_NONE = 2 };
/* Order of Alg. 1: the parallel form of §III.D (every non-negative column solved from the
 * outset; canonical) or the serial form of §III.C (donors solved after they donate). */
enum { O_REDREC_PARALLEL = 0, O_REDREC_SERIAL = 1, O_BIRD = 2 };

typedef struct { uint16_t w, h, x0, y0, x1, y1; } o_shape;
typedef struct { uint16_t sx, sy, dx, dy; } o_move;
typedef struct { int32_t status; uint32_t n_moves, n_groups, n_steps, need_moves, need_groups; } o_solve_info;
typedef struct { int32_t status; uint32_t n_batches, n_steps, need_batches, need_steps; } o_batch_info;
/* One iteration of the donor/receiver loop: donor i, receiver j, case 1..3, tokens taken from
 * the donor's lower reservoir (k, case 1-2 only) and total tokens handed over. */
typedef struct { int32_t donor, receiver, kase, k_bottom, count; } o_event;

#define MAX_SIDE 1024

static int iabs(int v) { return v < 0 ? -v : v; }
static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }

static int shape_ok(const o_shape *s)
{
    if (!s) return 0;
    if (s->w < 1 || s->h < 1 || s->w > MAX_SIDE || s->h > MAX_SIDE) return 0;
    if (!(s->x0 < s->x1 && s->x1 <= s->w)) return 0;
    if (!(s->y0 < s->y1 && s->y1 <= s->h)) return 0;
    return 1;
}

/* ---------------------------------------------------------------------------------------- */
/* growable move list with group boundaries                                                 */

typedef struct {
    o_move *m; size_t n, cap;
    uint32_t *goff; size_t ng, gcap;   /* goff[0..ng] */
    int oom;
} mlist;

static void ml_init(mlist *L)
{
    memset(L, 0, sizeof *L);
    L->gcap = 64;
    L->goff = (uint32_t *)malloc(L->gcap * sizeof(uint32_t));
    if (!L->goff) { L->oom = 1; return; }
    L->goff[0] = 0;
}

static void ml_free(mlist *L) { free(L->m); free(L->goff); }

static void ml_push(mlist *L, int sx, int sy, int dx, int dy)
{
    if (L->oom) return;
    if (L->n == L->cap) {
        size_t nc = L->cap ? 2 * L->cap : 256;
        o_move *nm = (o_move *)realloc(L->m, nc * sizeof(o_move));
        if (!nm) { L->oom = 1; return; }
        L->m = nm; L->cap = nc;
    }
    L->m[L->n].sx = (uint16_t)sx; L->m[L->n].sy = (uint16_t)sy;
    L->m[L->n].dx = (uint16_t)dx; L->m[L->n].dy = (uint16_t)dy;
    L->n++;
}

/* Close the group that began at move index `start`; an empty group is dropped. */
static void ml_close_group(mlist *L, size_t start)
{
    if (L->oom || L->n == start) return;
    if (L->ng + 2 > L->gcap) {
        size_t nc = 2 * L->gcap;
        uint32_t *ng = (uint32_t *)realloc(L->goff, nc * sizeof(uint32_t));
        if (!ng) { L->oom = 1; return; }
        L->goff = ng; L->gcap = nc;
    }
    L->ng++;
    L->goff[L->ng] = (uint32_t)L->n;
}

/* Execute moves [from, L->n) on the dense grid in list order. */
static void apply_moves(unsigned char *cell, int W, const mlist *L, size_t from)
{
    for (size_t b = from; b < L->n; ++b) {
        cell[L->m[b].sy * W + L->m[b].sx] = 0;
        cell[L->m[b].dy * W + L->m[b].dx] = 1;
    }
}

/* ---------------------------------------------------------------------------------------- */
/* Exact 1D (§III.A)                                                                       */

/* Assignment on a path with a contiguous target (§III.A, "Assignment").  Sources p[0..a) are
 * sorted and distinct, the targets are the t cells b, b+1, ..., b+t-1, and a >= t.  A
 * distance-minimising matching that saturates the targets can be taken order-preserving on a
 * run of t consecutive sorted sources, so the matching is fixed by the start w of that run:
 * cost(w) = sum_k |p[w+k] - (b+k)|.  Every w is tried; the smallest cost wins and, on equal
 * cost, the leftmost run (reading: the paper does not fix a tie rule). */
static int e1d_window(const int *p, int a, int b, int t)
{
    long best = -1;
    int best_w = 0;
    for (int w = 0; w + t <= a; ++w) {
        long c = 0;
        for (int k = 0; k < t; ++k) c += iabs(p[w + k] - (b + k));
        if (best < 0 || c < best) { best = c; best_w = w; }
    }
    return best_w;
}

/* Move generation on a line (§III.A, "Generating moves").  The matched pairs src[k] -> tgt[k]
 * (both increasing in k) become paths along the line.  Paths running towards larger
 * coordinates ("right-oriented") go first, from the one with the largest target down; then the
 * paths towards smaller coordinates, from the smallest target up; a source that is already its
 * target gives no move.  `horizontal` selects a row (fixed = y) or a column (fixed = x). */
static void emit_line(mlist *L, int horizontal, int fixed, const int *src, const int *tgt, int n)
{
    for (int k = n - 1; k >= 0; --k)
        if (src[k] < tgt[k]) {
            if (horizontal) ml_push(L, src[k], fixed, tgt[k], fixed);
            else            ml_push(L, fixed, src[k], fixed, tgt[k]);
        }
    for (int k = 0; k < n; ++k)
        if (src[k] > tgt[k]) {
            if (horizontal) ml_push(L, src[k], fixed, tgt[k], fixed);
            else            ml_push(L, fixed, src[k], fixed, tgt[k]);
        }
}

/* exported for the exact-1D tests: window start, or -1 on bad arguments */
int rr_oracle_e1d_window(const int *p, int a, int b, int t)
{
    if (!p || t < 0 || a < t) return -1;
    return e1d_window(p, a, b, t);
}

/* exported for the exact-1D tests: emitted moves of one line as (src, dst) pairs, in order */
int rr_oracle_e1d_moves(const int *p, int a, int b, int t, int *out_src, int *out_dst)
{
    if (!p || t < 0 || a < t) return -1;
    int w = e1d_window(p, a, b, t);
    int *src = (int *)malloc(sizeof(int) * (size_t)(t > 0 ? t : 1));
    int *tgt = (int *)malloc(sizeof(int) * (size_t)(t > 0 ? t : 1));
    mlist L; ml_init(&L);
    if (!src || !tgt || L.oom) { free(src); free(tgt); ml_free(&L); return -1; }
    for (int k = 0; k < t; ++k) { src[k] = p[w + k]; tgt[k] = b + k; }
    emit_line(&L, 1, 0, src, tgt, t);
    int n = (int)L.n;
    for (int i = 0; i < n; ++i) { out_src[i] = L.m[i].sx; out_dst[i] = L.m[i].dx; }
    free(src); free(tgt); ml_free(&L);
    return n;
}

/* ---------------------------------------------------------------------------------------- */
/* red-rec (Alg. 1, with the parallel-variant order of §III.D)                              */

typedef struct { int y, origin; long key; } o_src;

static int cmp_src(const void *a, const void *b)
{
    long ka = ((const o_src *)a)->key, kb = ((const o_src *)b)->key;
    return (ka > kb) - (ka < kb);
}

static int cmp_int(const void *a, const void *b)
{
    int ia = *(const int *)a, ib = *(const int *)b;
    return (ia > ib) - (ia < ib);
}

typedef struct {
    int W, H, x0, y0, x1, y1, sw, sh;
    unsigned char *cell;       /* cell[y*W + x] */
    int *q, *na;               /* q[x*H + k]: sorted eligible rows of column x; na[x] = count */
    int *sigma, *sp;           /* surplus, and the surplus seen by the pair loop */
    int *bp, *nb, *bh;         /* lower reservoir pool of column x, nearest-first; size; head */
    int *up, *nu, *uh;         /* upper reservoir pool of column x, nearest-first; size; head */
    o_src *mk; int *nm;        /* tokens marked for receiver x (row, donor); count */
    int serial;                /* serial order of Alg. 1 (donors solved after they donate) */
    int bird;                  /* bird (Alg. 2) instead of the donor/receiver loop */
    int *solved;               /* central column already solved (serial order) */
    int *dr;                   /* scratch rows of a donor solve */
    mlist L;
    o_event *ev; uint32_t ev_cap, n_ev;
    int status;
} rr_state;

/* Key for sorting the sources of a receiver solve: by row, and among tokens standing in the
 * same row (they come from different columns), the token that reaches the receiver column
 * first -- its own token, then the nearer donor, then the left donor -- takes the target that
 * lies farther from that row (reading: the paper leaves the order of such tokens open).
 * h = |origin - j| * W + origin grows with horizontal distance; above the band the farther
 * target is the lower one (sorted first), below the band it is the higher one (sorted last). */
static long source_key(const rr_state *S, int j, int y, int origin)
{
    long h = (long)iabs(origin - j) * S->W + origin;
    long tau = (y >= S->y1) ? h : (y < S->y0 ? -h : 0);
    return (long)y * 4L * S->W * S->W + tau;
}

/* Solve receiver column j (§III.C, redistribution cast as exact 1D; §III.D): its own tokens,
 * every token marked for it, and the tokens just chosen from its final donor -- exactly sh of
 * them -- are matched in row order to the band rows of column j.  A redistributed token runs
 * along its own row to column j, then along column j (reading: the paper drops the common
 * horizontal distance and leaves the route open).  Moves follow the exact-1D emission order. */
static void solve_receiver(rr_state *S, int j, const o_src *chosen, int n_chosen)
{
    int n = S->na[j] + S->nm[j] + n_chosen;
    o_src *s = (o_src *)malloc(sizeof(o_src) * (size_t)(n > 0 ? n : 1));
    if (!s) { S->L.oom = 1; return; }
    int c = 0;
    for (int k = 0; k < S->na[j]; ++k) { s[c].y = S->q[j * S->H + k]; s[c].origin = j; c++; }
    for (int k = 0; k < S->nm[j]; ++k) s[c++] = S->mk[(size_t)j * S->H + k];
    for (int k = 0; k < n_chosen; ++k) s[c++] = chosen[k];
    for (int k = 0; k < n; ++k) s[k].key = source_key(S, j, s[k].y, s[k].origin);
    qsort(s, (size_t)n, sizeof(o_src), cmp_src);
    if (n != S->sh) { S->status = O_E_INTERNAL; free(s); return; }

    size_t start = S->L.n;
    for (int k = n - 1; k >= 0; --k)          /* towards larger rows, largest target first */
        if (s[k].y < S->y0 + k || (s[k].y == S->y0 + k && s[k].origin != j))
            ml_push(&S->L, s[k].origin, s[k].y, j, S->y0 + k);
    for (int k = 0; k < n; ++k)               /* towards smaller rows, smallest target first */
        if (s[k].y > S->y0 + k)
            ml_push(&S->L, s[k].origin, s[k].y, j, S->y0 + k);
    apply_moves(S->cell, S->W, &S->L, start);
    ml_close_group(&S->L, start);
    free(s);
}

/* Summed distance of the receiver's 1-D problem when the chosen set takes the k nearest lower
 * tokens and the d-k nearest upper tokens of donor i: the sources (own, marked, chosen) are
 * sorted and matched in order to the band rows y0, y0+1, ... (§III.C: receiver target plus
 * donor reservoir as one line). */
static long split_cost(const rr_state *S, int i, int j, int k, int d, int *rows)
{
    int c = 0;
    for (int m = 0; m < S->na[j]; ++m) rows[c++] = S->q[j * S->H + m];
    for (int m = 0; m < S->nm[j]; ++m) rows[c++] = S->mk[(size_t)j * S->H + m].y;
    for (int m = 0; m < k; ++m) rows[c++] = S->bp[i * S->H + S->bh[i] + m];
    for (int m = 0; m < d - k; ++m) rows[c++] = S->up[i * S->H + S->uh[i] + m];
    qsort(rows, (size_t)c, sizeof(int), cmp_int);
    long cost = 0;
    for (int m = 0; m < c; ++m) cost += iabs(rows[m] - (S->y0 + m));
    return cost;
}

/* Solve donor column x in the serial order of Alg. 1 (its case 2 and case 3, and the columns
 * still unsolved when the loop ends): exact 1D onto [y0, y1) over the tokens the column still
 * holds -- its band tokens and what is left of its reservoir pool (the rest was handed to
 * earlier receivers).  The unmatched tokens lie outside the band (exact-1D lemma) and become
 * the column's pool again, nearest to the band first. */
static void solve_donor(rr_state *S, int x)
{
    const int H = S->H, y0 = S->y0, y1 = S->y1, sh = S->sh;
    int *r = S->dr, a = 0;
    for (int m = S->nb[x] - 1; m >= S->bh[x]; --m) r[a++] = S->bp[x * H + m];   /* below, ascending */
    for (int k = 0; k < S->na[x]; ++k) {
        int y = S->q[x * H + k];
        if (y >= y0 && y < y1) r[a++] = y;
    }
    for (int m = S->uh[x]; m < S->nu[x]; ++m) r[a++] = S->up[x * H + m];          /* above, ascending */
    if (a < sh) { S->status = O_E_INTERNAL; return; }
    int w = e1d_window(r, a, y0, sh);
    int *src = (int *)malloc(sizeof(int) * (size_t)sh), *tgt = (int *)malloc(sizeof(int) * (size_t)sh);
    if (!src || !tgt) { free(src); free(tgt); S->L.oom = 1; return; }
    for (int k = 0; k < sh; ++k) { src[k] = r[w + k]; tgt[k] = y0 + k; }
    size_t start = S->L.n;
    emit_line(&S->L, 0, x, src, tgt, sh);
    apply_moves(S->cell, S->W, &S->L, start);
    ml_close_group(&S->L, start);
    free(src); free(tgt);
    S->nb[x] = S->bh[x] = S->nu[x] = S->uh[x] = 0;
    for (int k = w - 1; k >= 0; --k) S->bp[x * H + S->nb[x]++] = r[k];
    for (int k = w + sh; k < a; ++k) S->up[x * H + S->nu[x]++] = r[k];
    S->solved[x] = 1;
}

/* Is pair (i, j) better than (bi, bj) under the pairing rule (§III.C): more tokens exchanged
 * (min of donor surplus and receiver deficit), then fewer columns in between, then the
 * receiver closer to saturation, then (reading: the paper stops there) the smaller receiver
 * index, then the smaller donor index. */
static int pair_better(const int *sp, int i, int j, int bi, int bj)
{
    int m = imin(sp[i], -sp[j]), bm = imin(sp[bi], -sp[bj]);
    if (m != bm) return m > bm;
    int dd = iabs(i - j), bd = iabs(bi - bj);
    if (dd != bd) return dd < bd;
    if (-sp[j] != -sp[bj]) return -sp[j] < -sp[bj];
    if (j != bj) return j < bj;
    return i < bi;
}

/* A token of the generalized 1-D instance of bird: virtual row v on the column being solved,
 * tie order t among tokens of one virtual row, physical trap (x, y). */
typedef struct { int v, t, x, y; } o_vtok;

static int cmp_vtok(const void *a, const void *b)
{
    const o_vtok *p = (const o_vtok *)a, *q = (const o_vtok *)b;
    if (p->v != q->v) return (p->v > q->v) - (p->v < q->v);
    return (p->t > q->t) - (p->t < q->t);
}

/* bird (§III.E, Alg. 2) after the non-negative columns are solved: the columns of negative
 * surplus, leftmost first, each filled by the generalized exact 1D.  For column j the line is
 * column j itself; its own tokens stand at their rows, and every reservoir token of another
 * column x stands at the row it would reach with the same Manhattan distance to the target of
 * column j: y + |x - j| above the band, y - |x - j| below it (several tokens can share one
 * virtual row; target rows of other columns are never taken).  The generalized exact 1D (the
 * cheapest run of sh consecutive sorted virtual tokens, ties to the leftmost run) picks the
 * tokens; among tokens of one virtual row the nearest column comes first, and on equal
 * distance the left column (reading: the paper fixes only "the closest possible column"), so a
 * run boundary inside a shared row keeps the nearest tokens.  A chosen token runs along its
 * row to column j, then along the column; moves follow the exact-1D emission order. */
static void bird(rr_state *S)
{
    const int W = S->W, H = S->H, x0 = S->x0, y0 = S->y0, x1 = S->x1, y1 = S->y1, sh = S->sh;
    o_vtok *c = (o_vtok *)malloc(sizeof(o_vtok) * (size_t)W * H);
    int *v = (int *)malloc(sizeof(int) * (size_t)W * H);
    if (!c || !v) { free(c); free(v); S->L.oom = 1; return; }
    for (int j = x0; j < x1; ++j) {
        if (S->sigma[j] >= 0) continue;
        int n = 0;
        for (int x = 0; x < W; ++x)
            for (int y = 0; y < H; ++y) {
                if (!S->cell[y * W + x]) continue;
                int band = (y >= y0 && y < y1);
                if (x != j && band) continue;
                int d = iabs(x - j), pr = 2 * d + (x > j);
                c[n].x = x; c[n].y = y;
                c[n].v = (x == j) ? y : (y >= y1 ? y + d : y - d);
                c[n].t = (c[n].v >= y0) ? pr : -pr;     /* nearest first above, nearest last below */
                n++;
            }
        if (n < sh) { S->status = O_E_INTERNAL; break; }
        qsort(c, (size_t)n, sizeof(o_vtok), cmp_vtok);
        for (int k = 0; k < n; ++k) v[k] = c[k].v;
        int w = e1d_window(v, n, y0, sh);
        size_t start = S->L.n;
        for (int k = sh - 1; k >= 0; --k)                 /* towards larger rows, largest target first */
            if (c[w + k].v < y0 + k) ml_push(&S->L, c[w + k].x, c[w + k].y, j, y0 + k);
        for (int k = 0; k < sh; ++k)                      /* towards smaller rows, smallest target first */
            if (c[w + k].v > y0 + k) ml_push(&S->L, c[w + k].x, c[w + k].y, j, y0 + k);
        apply_moves(S->cell, W, &S->L, start);
        ml_close_group(&S->L, start);
    }
    free(c); free(v);
}

static void redrec(rr_state *S)
{
    const int W = S->W, H = S->H, x0 = S->x0, y0 = S->y0, x1 = S->x1, y1 = S->y1;
    const int sw = S->sw, sh = S->sh;
    int *p = (int *)malloc(sizeof(int) * (size_t)(W > H ? W : H));
    int *src = (int *)malloc(sizeof(int) * (size_t)(W > H ? W : H));
    int *tgt = (int *)malloc(sizeof(int) * (size_t)(W > H ? W : H));
    int *rows = (int *)malloc(sizeof(int) * (size_t)(H + 1));
    o_src *chosen = (o_src *)malloc(sizeof(o_src) * (size_t)(H + 1));
    if (!p || !src || !tgt || !rows || !chosen) { S->L.oom = 1; goto out; }

    /* Feasibility.  N tokens; when side columns exist, band-row tokens beyond sw per row stay
     * parked in side columns and never count.  The instance is solved iff
     * F = N - D - sw*sh >= 0 (reading: with side columns the paper gives no rule; for a
     * full-width band this is |S| >= |T|, §II.B). */
    int side = (x0 > 0 || x1 < W);
    long N = 0, D = 0;
    for (int i = 0; i < W * H; ++i) N += S->cell[i];
    if (side)
        for (int y = y0; y < y1; ++y) {
            int a = 0;
            for (int x = 0; x < W; ++x) a += S->cell[y * W + x];
            D += imax(0, a - sw);
        }
    if (N - D - (long)sw * sh < 0) { S->status = O_INFEASIBLE; goto out; }

    /* Stage H (reading: the paper's red-rec assumes a band spanning every column and leaves
     * other targets open).  Each band row is first solved on its own line: with at least sw
     * tokens, exact 1D onto [x0, x1) (the unmatched tokens lie outside the target and stay,
     * parked); with fewer, the tokens are packed in order onto the centred run
     * [c, c + a), c = x0 + floor((sw - a) / 2).  One group per row, rows in ascending order. */
    if (side)
        for (int y = y0; y < y1; ++y) {
            int a = 0;
            for (int x = 0; x < W; ++x) if (S->cell[y * W + x]) p[a++] = x;
            int n;
            if (a >= sw) {
                int w = e1d_window(p, a, x0, sw);
                for (int k = 0; k < sw; ++k) { src[k] = p[w + k]; tgt[k] = x0 + k; }
                n = sw;
            } else {
                int c = x0 + (sw - a) / 2;
                for (int k = 0; k < a; ++k) { src[k] = p[k]; tgt[k] = c + k; }
                n = a;
            }
            size_t start = S->L.n;
            emit_line(&S->L, 1, y, src, tgt, n);
            apply_moves(S->cell, W, &S->L, start);
            ml_close_group(&S->L, start);
        }

    /* Surplus (Alg. 1): sigma_x = |S n C_x| - |T n C_x|.  A central column counts every
     * token; a side column has no target and counts only its reservoir-row tokens (the
     * parked band tokens are not available). */
    for (int x = 0; x < W; ++x) {
        int central = (x >= x0 && x < x1);
        int a = 0;
        for (int y = 0; y < H; ++y)
            if (S->cell[y * W + x] && (central || y < y0 || y >= y1)) S->q[x * H + a++] = y;
        S->na[x] = a;
        S->sigma[x] = a - (central ? sh : 0);
    }

    /* Columns with non-negative surplus are solved from the outset, in ascending x (§III.D).
     * A central one is solved by exact 1D onto [y0, y1); its unmatched tokens stay where they
     * are and form its donor pool: B below the band, nearest first, and U above it, nearest
     * first.  A side column has nothing to solve; its reservoir tokens form its pool.
     * Serial order (Alg. 1 as written): only the columns of zero surplus are solved here; a
     * central donor keeps all its tokens until it is solved, and its pool is its reservoir
     * tokens, nearest to the band first. */
    for (int x = 0; x < W; ++x) {
        S->nb[x] = S->nu[x] = S->bh[x] = S->uh[x] = S->nm[x] = 0;
        S->solved[x] = 0;
        if (S->sigma[x] < 0) continue;
        const int *qx = S->q + x * H;
        int a = S->na[x];
        if (x >= x0 && x < x1 && S->serial && S->sigma[x] > 0) {
            for (int k = a - 1; k >= 0; --k) if (qx[k] < y0) S->bp[x * H + S->nb[x]++] = qx[k];
            for (int k = 0; k < a; ++k) if (qx[k] >= y1) S->up[x * H + S->nu[x]++] = qx[k];
        } else if (x >= x0 && x < x1) {
            S->solved[x] = 1;
            int w = e1d_window(qx, a, y0, sh);
            for (int k = 0; k < sh; ++k) { src[k] = qx[w + k]; tgt[k] = y0 + k; }
            size_t start = S->L.n;
            emit_line(&S->L, 0, x, src, tgt, sh);
            apply_moves(S->cell, W, &S->L, start);
            ml_close_group(&S->L, start);
            for (int k = w - 1; k >= 0; --k) S->bp[x * H + S->nb[x]++] = qx[k];
            for (int k = w + sh; k < a; ++k) S->up[x * H + S->nu[x]++] = qx[k];
        } else {
            for (int k = a - 1; k >= 0; --k) if (qx[k] < y0) S->bp[x * H + S->nb[x]++] = qx[k];
            for (int k = 0; k < a; ++k) if (qx[k] >= y1) S->up[x * H + S->nu[x]++] = qx[k];
        }
    }

    if (S->bird) { bird(S); goto out; }

    /* Donor/receiver loop (Alg. 1 main loop, pairing rule of §III.C).  sp = pool size for a
     * solved column, the deficit for a receiver (negative), 0 once a column is settled. */
    for (int x = 0; x < W; ++x) S->sp[x] = S->sigma[x];
    for (;;) {
        int any_neg = 0;
        for (int x = 0; x < W; ++x) if (S->sp[x] < 0) any_neg = 1;
        if (!any_neg) break;

        /* Candidate pairs: a donor and a receiver with only settled columns between them,
         * i.e. consecutive entries of opposite sign among the unsettled columns. */
        int bi = -1, bj = -1, prev = -1;
        for (int x = 0; x < W; ++x) {
            if (S->sp[x] == 0) continue;
            if (prev >= 0 && ((S->sp[prev] > 0) != (S->sp[x] > 0))) {
                int i = S->sp[prev] > 0 ? prev : x;
                int j = S->sp[prev] > 0 ? x : prev;
                if (bi < 0 || pair_better(S->sp, i, j, bi, bj)) { bi = i; bj = j; }
            }
            prev = x;
        }
        if (bi < 0) { S->status = O_E_INTERNAL; goto out; }
        int i = bi, j = bj;
        int avail = S->nb[i] - S->bh[i] + S->nu[i] - S->uh[i];
        int d = -S->sp[j];
        int unsolved = (i >= x0 && i < x1 && !S->solved[i]);   /* serial order only */
        if (unsolved ? avail < S->sp[i] : avail != S->sp[i]) { S->status = O_E_INTERNAL; goto out; }

        if (S->sp[i] < d) {
            /* Case 3: the donor's whole pool is marked for the receiver; nothing moves yet.  In
             * the serial order the donor is solved first, and its pool is then its excess. */
            if (unsolved) {
                solve_donor(S, i);
                if (S->status != O_OK || S->L.oom) goto out;
            }
            int cnt = 0;
            for (int m = S->bh[i]; m < S->nb[i]; ++m) {
                o_src t; t.y = S->bp[i * H + m]; t.origin = i; t.key = 0;
                S->mk[(size_t)j * H + S->nm[j]++] = t; cnt++;
            }
            for (int m = S->uh[i]; m < S->nu[i]; ++m) {
                o_src t; t.y = S->up[i * H + m]; t.origin = i; t.key = 0;
                S->mk[(size_t)j * H + S->nm[j]++] = t; cnt++;
            }
            S->bh[i] = S->nb[i]; S->uh[i] = S->nu[i];
            S->sp[j] += S->sp[i];
            S->sp[i] = 0;
            if (S->ev && S->n_ev < S->ev_cap) {
                o_event e = { i, j, 3, -1, cnt };
                S->ev[S->n_ev] = e;
            }
            S->n_ev++;
        } else {
            /* Cases 1 and 2: the donor saturates the receiver.  The d tokens taken are the
             * k nearest below the band and the d-k nearest above it, with k minimising the
             * receiver's 1-D cost; on equal cost the largest k. */
            int bav = S->nb[i] - S->bh[i], uav = S->nu[i] - S->uh[i];
            int klo = imax(0, d - uav), khi = imin(d, bav);
            long best = -1; int bk = klo;
            for (int k = klo; k <= khi; ++k) {
                long c = split_cost(S, i, j, k, d, rows);
                if (best < 0 || c <= best) { best = c; bk = k; }
            }
            int nc = 0;
            for (int m = 0; m < bk; ++m) {
                chosen[nc].y = S->bp[i * H + S->bh[i] + m]; chosen[nc].origin = i; nc++;
            }
            for (int m = 0; m < d - bk; ++m) {
                chosen[nc].y = S->up[i * H + S->uh[i] + m]; chosen[nc].origin = i; nc++;
            }
            S->bh[i] += bk; S->uh[i] += d - bk;
            int kase = (S->sp[i] == d) ? 2 : 1;
            S->sp[i] -= d;
            S->sp[j] = 0;
            if (S->ev && S->n_ev < S->ev_cap) {
                o_event e = { i, j, kase, bk, d };
                S->ev[S->n_ev] = e;
            }
            S->n_ev++;
            solve_receiver(S, j, chosen, nc);
            if (S->status != O_OK) goto out;
            /* Case 2 in the serial order: the donor, left with exactly sh tokens, is solved
             * right after the receiver. */
            if (kase == 2 && unsolved) {
                solve_donor(S, i);
                if (S->status != O_OK || S->L.oom) goto out;
            }
        }
    }
    /* Serial order: the columns still unsolved when every receiver is saturated are solved
     * last, in ascending x; their excess stays in the reservoir. */
    if (S->serial)
        for (int x = x0; x < x1; ++x)
            if (!S->solved[x] && S->sigma[x] > 0) {
                solve_donor(S, x);
                if (S->status != O_OK || S->L.oom) goto out;
            }
out:
    free(p); free(src); free(tgt); free(rows); free(chosen);
}

static int solve_impl(const o_shape *shape, const uint64_t *occ, o_move *moves, uint32_t move_cap,
                      uint32_t *group_off, uint32_t group_cap, uint64_t *final_occ, o_solve_info *info,
                      uint32_t flags, o_event *ev, uint32_t ev_cap, uint32_t *n_ev)
{
    if (!shape_ok(shape) || !occ || !info || flags > O_BIRD) return O_E_INVAL;
    rr_state S;
    memset(&S, 0, sizeof S);
    S.serial = (flags == O_REDREC_SERIAL);
    S.bird = (flags == O_BIRD);
    S.W = shape->w; S.H = shape->h;
    S.x0 = shape->x0; S.y0 = shape->y0; S.x1 = shape->x1; S.y1 = shape->y1;
    S.sw = S.x1 - S.x0; S.sh = S.y1 - S.y0;
    S.ev = ev; S.ev_cap = ev_cap;
    const int W = S.W, H = S.H, ws = (W + 63) / 64;
    size_t WH = (size_t)W * H;
    S.cell = (unsigned char *)calloc(WH, 1);
    S.q = (int *)malloc(sizeof(int) * WH);
    S.bp = (int *)malloc(sizeof(int) * WH);
    S.up = (int *)malloc(sizeof(int) * WH);
    S.mk = (o_src *)malloc(sizeof(o_src) * WH);
    S.na = (int *)calloc((size_t)W, sizeof(int));
    S.sigma = (int *)calloc((size_t)W, sizeof(int));
    S.sp = (int *)calloc((size_t)W, sizeof(int));
    S.nb = (int *)calloc((size_t)W, sizeof(int));
    S.bh = (int *)calloc((size_t)W, sizeof(int));
    S.nu = (int *)calloc((size_t)W, sizeof(int));
    S.uh = (int *)calloc((size_t)W, sizeof(int));
    S.nm = (int *)calloc((size_t)W, sizeof(int));
    S.solved = (int *)calloc((size_t)W, sizeof(int));
    S.dr = (int *)malloc(sizeof(int) * (size_t)(H + 1));
    ml_init(&S.L);
    int rc = O_OK;
    if (!S.cell || !S.q || !S.bp || !S.up || !S.mk || !S.na || !S.sigma || !S.sp || !S.nb || !S.bh ||
        !S.nu || !S.uh || !S.nm || !S.solved || !S.dr || S.L.oom) { rc = O_E_NOMEM; goto done; }

    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            S.cell[y * W + x] = (unsigned char)((occ[(size_t)y * ws + x / 64] >> (x % 64)) & 1u);

    S.status = O_OK;
    redrec(&S);
    if (S.L.oom) { rc = O_E_NOMEM; goto done; }
    if (n_ev) *n_ev = S.n_ev;

    memset(info, 0, sizeof *info);
    if (S.status == O_INFEASIBLE || S.status == O_E_INTERNAL) {
        info->status = S.status;
        info->need_moves = 0; info->need_groups = 0;
        if (group_off) group_off[0] = 0;
        goto write_final;                  /* no move was made: the final grid is the input */
    }
    uint64_t steps = 0;
    for (size_t b = 0; b < S.L.n; ++b)
        steps += (uint64_t)(iabs(S.L.m[b].dx - S.L.m[b].sx) + iabs(S.L.m[b].dy - S.L.m[b].sy));
    info->need_moves = (uint32_t)S.L.n;
    info->need_groups = (uint32_t)S.L.ng;
    if (S.L.n > move_cap || S.L.ng > group_cap || !group_off || (S.L.n && !moves)) {
        info->status = O_E_CAPACITY;
        goto done;
    }
    if (S.L.n) memcpy(moves, S.L.m, sizeof(o_move) * S.L.n);
    memcpy(group_off, S.L.goff, sizeof(uint32_t) * (S.L.ng + 1));
    info->status = O_OK;
    info->n_moves = (uint32_t)S.L.n;
    info->n_groups = (uint32_t)S.L.ng;
    info->n_steps = (uint32_t)steps;
write_final:
    if (final_occ) {
        memset(final_occ, 0, sizeof(uint64_t) * (size_t)H * ws);
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                if (S.cell[y * W + x]) final_occ[(size_t)y * ws + x / 64] |= (uint64_t)1 << (x % 64);
    }
done:
    free(S.cell); free(S.q); free(S.bp); free(S.up); free(S.mk);
    free(S.na); free(S.sigma); free(S.sp); free(S.nb); free(S.bh); free(S.nu); free(S.uh); free(S.nm);
    free(S.solved); free(S.dr);
    ml_free(&S.L);
    return rc;
}

/* Solve one instance.  group_off has room for group_cap + 1 entries; moves for move_cap. */
int rr_oracle_solve(const o_shape *shape, const uint64_t *occ, o_move *moves, uint32_t move_cap,
                    uint32_t *group_off, uint32_t group_cap, uint64_t *final_occ, o_solve_info *info)
{
    return solve_impl(shape, occ, moves, move_cap, group_off, group_cap, final_occ, info, O_REDREC_PARALLEL,
                      NULL, 0, NULL);
}

/* Same solve, also reporting the donor/receiver loop's events in order; flags selects the
 * order of Alg. 1 (O_REDREC_PARALLEL or O_REDREC_SERIAL) or bird (O_BIRD, no events). */
int rr_oracle_solve_trace(const o_shape *shape, const uint64_t *occ, o_move *moves, uint32_t move_cap,
                          uint32_t *group_off, uint32_t group_cap, uint64_t *final_occ, o_solve_info *info,
                          uint32_t flags, o_event *events, uint32_t event_cap, uint32_t *n_events)
{
    return solve_impl(shape, occ, moves, move_cap, group_off, group_cap, final_occ, info, flags,
                      events, event_cap, n_events);
}

/* ---------------------------------------------------------------------------------------- */
/* Batching (§IV, Alg. 3)                                                                  */

/* Cell s (0..len) of the path of move m: along row sy from sx to dx, then along column dx. */
static void path_cell(const o_move *m, int s, int *x, int *y)
{
    int hx = iabs((int)m->dx - (int)m->sx);
    if (s <= hx) {
        *x = (int)m->sx + (m->dx >= m->sx ? s : -s);
        *y = m->sy;
    } else {
        *x = m->dx;
        *y = (int)m->sy + (m->dy >= m->sy ? (s - hx) : -(s - hx));
    }
}

static int path_len(const o_move *m)
{
    return iabs((int)m->dx - (int)m->sx) + iabs((int)m->dy - (int)m->sy);
}

/* direction code of a unit step: 0 +x, 1 -x, 2 +y, 3 -y */
static int step_dir(int ux, int uy, int vx, int vy)
{
    if (vx > ux) return 0;
    if (vx < ux) return 1;
    if (vy > uy) return 2;
    return 3;
}

typedef struct { int ux, uy, vx, vy, dir; } o_step;

/* Local constraint of §IV ("constrained batching"), checked pairwise: the deployed rule
 * allows batches of tokens in one column (row) moving the same way.  Reading: two steps are
 * compatible when they move the same way and their current traps share a column or a row;
 * the "along" variant also asks that the shared line be the direction of motion; "none"
 * drops the constraint. */
static int lambda_ok(uint32_t flags, const o_step *e, const o_step *f)
{
    if (flags == O_LAMBDA_NONE) return 1;
    if (e->dir != f->dir) return 0;
    int vertical = (e->dir >= 2);
    if (flags == O_LAMBDA_ALONG)
        return vertical ? (e->ux == f->ux) : (e->uy == f->uy);
    return (e->ux == f->ux) || (e->uy == f->uy);
}

static int disjoint(const o_step *e, const o_step *f)
{
    if (e->ux == f->ux && e->uy == f->uy) return 0;
    if (e->ux == f->vx && e->uy == f->vy) return 0;
    if (e->vx == f->ux && e->vy == f->uy) return 0;
    if (e->vx == f->vx && e->vy == f->vy) return 0;
    return 1;
}

typedef struct { uint32_t *a; size_t n, cap; int oom; } u32vec;
static void uv_push(u32vec *v, uint32_t x)
{
    if (v->oom) return;
    if (v->n == v->cap) {
        size_t nc = v->cap ? 2 * v->cap : 64;
        uint32_t *na = (uint32_t *)realloc(v->a, nc * sizeof(uint32_t));
        if (!na) { v->oom = 1; return; }
        v->a = na; v->cap = nc;
    }
    v->a[v->n++] = x;
}

/* Batch the moves of one solve.  The dependency graph Gamma follows §IV: within a group (one
 * exact-1D line or one column solve) move a precedes move b (a < b) when their paths share a
 * trap; across groups, every move of an earlier group precedes every move of a later group
 * when the two groups share any trap.  Alg. 3 then runs literally: each iteration takes the
 * moves with no remaining predecessor, in ascending move index (reading: the order of this set
 * is left open), and greedily adds each one's next unit step when it shares no trap with the
 * steps already in the batch and satisfies the local constraint with each of them.  A finished
 * move leaves Gamma; moves it was blocking wait for the next iteration.  Every move must have
 * at least one step (a move whose source is its target is rejected as invalid input).
 * steps[] holds dir << 30 | x << 15 | y of each step's source trap, batch by batch. */
int rr_oracle_batch_moves(const o_shape *shape, const o_move *mv, const uint32_t *goff,
                          const o_solve_info *si, uint32_t flags, uint32_t *batch_off, uint32_t batch_cap,
                          uint32_t *steps, uint32_t step_cap, o_batch_info *bi)
{
    if (!shape_ok(shape) || !si || !bi || flags > O_LAMBDA_NONE) return O_E_INVAL;
    memset(bi, 0, sizeof *bi);
    const int W = shape->w, H = shape->h;
    if (si->status == O_INFEASIBLE || (si->status == O_OK && si->n_moves == 0)) {
        bi->status = O_OK; bi->need_batches = 0; bi->need_steps = 0;
        if (batch_off) batch_off[0] = 0;
        return O_OK;
    }
    if (si->status != O_OK || !mv || !goff) { bi->status = O_E_INVAL; return O_OK; }
    const uint32_t K = si->n_moves, G = si->n_groups;
    if (goff[0] != 0 || goff[G] != K) { bi->status = O_E_INVAL; return O_OK; }
    for (uint32_t g = 0; g < G; ++g) if (goff[g] > goff[g + 1]) { bi->status = O_E_INVAL; return O_OK; }
    for (uint32_t b = 0; b < K; ++b)
        if (mv[b].sx >= W || mv[b].dx >= W || mv[b].sy >= H || mv[b].dy >= H || path_len(&mv[b]) == 0) {
            bi->status = O_E_INVAL; return O_OK;
        }

    /* steps capacity first: without room for every step nothing is batched; need_batches is
     * then reported as the step count, an upper bound on the number of batches */
    uint64_t T = 0;
    for (uint32_t b = 0; b < K; ++b) T += (uint64_t)path_len(&mv[b]);
    if (T > step_cap) {
        bi->status = O_E_CAPACITY; bi->need_steps = (uint32_t)T; bi->need_batches = (uint32_t)T;
        return O_OK;
    }

    int rc = O_OK;
    size_t WH = (size_t)W * H, gw = (WH + 63) / 64;
    uint32_t *grp = (uint32_t *)malloc(sizeof(uint32_t) * K);
    int *len = (int *)malloc(sizeof(int) * K);
    int *pos = (int *)calloc(K, sizeof(int));
    int *alive = (int *)calloc(K, sizeof(int));
    int *indeg = (int *)calloc(K, sizeof(int));
    u32vec *succ = (u32vec *)calloc(K, sizeof(u32vec));
    uint64_t *gbits = (uint64_t *)calloc((size_t)G * gw, sizeof(uint64_t));
    u32vec *gpred = (u32vec *)calloc(G, sizeof(u32vec));
    int *gremain = (int *)calloc(G, sizeof(int));
    int *unlocked = (int *)calloc(G, sizeof(int));
    uint32_t *stamp = (uint32_t *)calloc(WH, sizeof(uint32_t));
    uint32_t *Q = (uint32_t *)malloc(sizeof(uint32_t) * K);
    o_step *B = (o_step *)malloc(sizeof(o_step) * K);
    u32vec outb = {0}, outs = {0};
    if (!grp || !len || !pos || !alive || !indeg || !succ || !gbits || !gpred || !gremain || !unlocked ||
        !stamp || !Q || !B) { rc = O_E_NOMEM; goto done; }

    for (uint32_t g = 0; g < G; ++g)
        for (uint32_t b = goff[g]; b < goff[g + 1]; ++b) grp[b] = g;
    for (uint32_t b = 0; b < K; ++b) len[b] = path_len(&mv[b]);

    /* group trap sets V(G) */
    for (uint32_t b = 0; b < K; ++b)
        for (int s = 0; s <= len[b]; ++s) {
            int x, y; path_cell(&mv[b], s, &x, &y);
            size_t c = (size_t)y * W + x;
            gbits[(size_t)grp[b] * gw + c / 64] |= (uint64_t)1 << (c % 64);
        }
    /* group-level edges: earlier group g precedes later group h when they share a trap */
    for (uint32_t h = 0; h < G; ++h)
        for (uint32_t g = 0; g < h; ++g) {
            int meet = 0;
            for (size_t k = 0; k < gw && !meet; ++k)
                if (gbits[(size_t)g * gw + k] & gbits[(size_t)h * gw + k]) meet = 1;
            if (meet) uv_push(&gpred[h], g);
        }
    /* move-level edges inside a group: a < b sharing a trap */
    uint32_t gen = 0;
    for (uint32_t g = 0; g < G; ++g)
        for (uint32_t b = goff[g]; b < goff[g + 1]; ++b) {
            for (uint32_t a = goff[g]; a < b; ++a) {
                ++gen;
                for (int s = 0; s <= len[a]; ++s) {
                    int x, y; path_cell(&mv[a], s, &x, &y);
                    stamp[(size_t)y * W + x] = gen;
                }
                int meet = 0;
                for (int s = 0; s <= len[b] && !meet; ++s) {
                    int x, y; path_cell(&mv[b], s, &x, &y);
                    if (stamp[(size_t)y * W + x] == gen) meet = 1;
                }
                if (meet) { uv_push(&succ[a], b); indeg[b]++; }
            }
        }
    for (uint32_t b = 0; b < K; ++b) if (succ[b].oom) { rc = O_E_NOMEM; goto done; }
    for (uint32_t g = 0; g < G; ++g) if (gpred[g].oom) { rc = O_E_NOMEM; goto done; }

    size_t n_alive = 0;
    for (uint32_t b = 0; b < K; ++b) {
        alive[b] = 1; gremain[grp[b]]++; n_alive++;
    }

    uv_push(&outb, 0);
    while (n_alive > 0) {
        /* Q: moves whose predecessors in Gamma have all left it */
        for (uint32_t h = 0; h < G; ++h) {
            unlocked[h] = 1;
            for (size_t e = 0; e < gpred[h].n; ++e) if (gremain[gpred[h].a[e]] > 0) unlocked[h] = 0;
        }
        size_t nq = 0;
        for (uint32_t b = 0; b < K; ++b)
            if (alive[b] && indeg[b] == 0 && unlocked[grp[b]]) Q[nq++] = b;
        size_t nbat = 0;
        for (size_t qi = 0; qi < nq; ++qi) {
            uint32_t b = Q[qi];
            o_step e;
            path_cell(&mv[b], pos[b], &e.ux, &e.uy);
            path_cell(&mv[b], pos[b] + 1, &e.vx, &e.vy);
            e.dir = step_dir(e.ux, e.uy, e.vx, e.vy);
            int ok = 1;
            for (size_t f = 0; f < nbat && ok; ++f)
                if (!disjoint(&e, &B[f]) || !lambda_ok(flags, &e, &B[f])) ok = 0;
            if (!ok) continue;
            B[nbat++] = e;
            uv_push(&outs, ((uint32_t)e.dir << 30) | ((uint32_t)e.ux << 15) | (uint32_t)e.uy);
            pos[b]++;
            if (pos[b] == len[b]) {
                alive[b] = 0; n_alive--; gremain[grp[b]]--;
                for (size_t s = 0; s < succ[b].n; ++s) indeg[succ[b].a[s]]--;
            }
        }
        if (nbat == 0) { rc = O_OK; bi->status = O_E_INTERNAL; goto done; }
        uv_push(&outb, (uint32_t)outs.n);
        if (outb.oom || outs.oom) { rc = O_E_NOMEM; goto done; }
    }

    bi->need_batches = (uint32_t)(outb.n - 1);
    bi->need_steps = (uint32_t)outs.n;
    if (outb.n - 1 > batch_cap || outs.n > step_cap || !batch_off || (outs.n && !steps)) {
        bi->status = O_E_CAPACITY;
        goto done;
    }
    memcpy(batch_off, outb.a, sizeof(uint32_t) * outb.n);
    if (outs.n) memcpy(steps, outs.a, sizeof(uint32_t) * outs.n);
    bi->status = O_OK;
    bi->n_batches = (uint32_t)(outb.n - 1);
    bi->n_steps = (uint32_t)outs.n;
done:
    if (succ) for (uint32_t b = 0; b < K; ++b) free(succ[b].a);
    if (gpred) for (uint32_t g = 0; g < G; ++g) free(gpred[g].a);
    free(grp); free(len); free(pos); free(alive); free(indeg); free(succ); free(gbits); free(gpred);
    free(gremain); free(unlocked); free(stamp); free(Q); free(B); free(outb.a); free(outs.a);
    return rc;
}

/* ---------------------------------------------------------------------------------------- */
/* Batching, indexed form: the same Alg. 3 for instances far beyond what the literal form    */
/* above can run (a 1024 x 1024 shot has ~6e5 moves and ~1e8 unit steps).                  */
/*                                                                                          */
/* Semantics are those of rr_oracle_batch_moves; only the bookkeeping differs:              */
/*  - Gamma is kept reduced.  A move waits on the previous toucher of each trap of its path */
/*    within its group, and a group on the previous group touching each of its traps.  The  */
/*    full relation follows by transitivity: the touchers of one trap are chained in index  */
/*    (group) order, so the last one having finished (completed) implies every earlier one  */
/*    has, and readiness is unchanged.                                                      */
/*  - The ready moves are kept in ascending index, and bucketed by (direction of the next   */
/*    step, row) and (direction, column) of their current trap.  Each iteration's Q is the  */
/*    ready set at its start (all updates wait until the batch is formed).  The first move  */
/*    of Q always enters the batch; under the line-or-column constraint every other step    */
/*    that could join it moves the same way on the first one's row or column, and once a   */
/*    second step has joined, the line it shares with the first is the only one left (a     */
/*    step compatible with both members yet off that line would stand on the first one's    */
/*    trap), so scanning the two buckets in index order visits exactly the candidates the   */
/*    literal scan of Q would accept.  Under "along" the one bucket of the motion's line is */
/*    scanned; without constraint the whole of Q.  Trap disjointness is tested as stated.   */
/* The two forms are checked equal on fixtures and random instances by the tests.           */

typedef struct { uint32_t *a; uint32_t n, cap; } sarr;     /* ascending move indices */

static int sa_find(const sarr *s, uint32_t v)
{
    uint32_t lo = 0, hi = s->n;
    while (lo < hi) { uint32_t m = (lo + hi) / 2; if (s->a[m] < v) lo = m + 1; else hi = m; }
    return (int)lo;
}

static int sa_insert(sarr *s, uint32_t v)
{
    if (s->n == s->cap) {
        uint32_t nc = s->cap ? 2 * s->cap : 8;
        uint32_t *na = (uint32_t *)realloc(s->a, nc * sizeof(uint32_t));
        if (!na) return 0;
        s->a = na; s->cap = nc;
    }
    int k = sa_find(s, v);
    memmove(s->a + k + 1, s->a + k, (s->n - (uint32_t)k) * sizeof(uint32_t));
    s->a[k] = v; s->n++;
    return 1;
}

static void sa_remove(sarr *s, uint32_t v)
{
    int k = sa_find(s, v);
    if ((uint32_t)k < s->n && s->a[k] == v) {
        memmove(s->a + k, s->a + k + 1, (s->n - (uint32_t)k - 1) * sizeof(uint32_t));
        s->n--;
    }
}

typedef struct {
    const o_move *mv;
    int W, H;
    int *pos, *len;
    uint8_t *rdir; uint16_t *rx, *ry;      /* bucket keys of a ready move */
    sarr ready, *rowb, *colb;              /* rowb[dir*H + y], colb[dir*W + x] */
    int oom;
} ix_state;

static void ix_step(const ix_state *X, uint32_t b, o_step *e)
{
    path_cell(&X->mv[b], X->pos[b], &e->ux, &e->uy);
    path_cell(&X->mv[b], X->pos[b] + 1, &e->vx, &e->vy);
    e->dir = step_dir(e->ux, e->uy, e->vx, e->vy);
}

static void ix_make_ready(ix_state *X, uint32_t b)
{
    o_step e;
    ix_step(X, b, &e);
    X->rdir[b] = (uint8_t)e.dir; X->rx[b] = (uint16_t)e.ux; X->ry[b] = (uint16_t)e.uy;
    if (!sa_insert(&X->ready, b) || !sa_insert(&X->rowb[e.dir * X->H + e.uy], b) ||
        !sa_insert(&X->colb[e.dir * X->W + e.ux], b))
        X->oom = 1;
}

static void ix_unready(ix_state *X, uint32_t b)
{
    sa_remove(&X->ready, b);
    sa_remove(&X->rowb[X->rdir[b] * X->H + X->ry[b]], b);
    sa_remove(&X->colb[X->rdir[b] * X->W + X->rx[b]], b);
}

int rr_oracle_batch_moves_indexed(const o_shape *shape, const o_move *mv, const uint32_t *goff,
                                  const o_solve_info *si, uint32_t flags, uint32_t *batch_off, uint32_t batch_cap,
                                  uint32_t *steps, uint32_t step_cap, o_batch_info *bi)
{
    if (!shape_ok(shape) || !si || !bi || flags > O_LAMBDA_NONE) return O_E_INVAL;
    memset(bi, 0, sizeof *bi);
    const int W = shape->w, H = shape->h;
    if (si->status == O_INFEASIBLE || (si->status == O_OK && si->n_moves == 0)) {
        bi->status = O_OK;
        if (batch_off) batch_off[0] = 0;
        return O_OK;
    }
    if (si->status != O_OK || !mv || !goff) { bi->status = O_E_INVAL; return O_OK; }
    const uint32_t K = si->n_moves, G = si->n_groups;
    if (goff[0] != 0 || goff[G] != K) { bi->status = O_E_INVAL; return O_OK; }
    for (uint32_t g = 0; g < G; ++g) if (goff[g] > goff[g + 1]) { bi->status = O_E_INVAL; return O_OK; }
    for (uint32_t b = 0; b < K; ++b)
        if (mv[b].sx >= W || mv[b].dx >= W || mv[b].sy >= H || mv[b].dy >= H || path_len(&mv[b]) == 0) {
            bi->status = O_E_INVAL; return O_OK;
        }
    uint64_t T = 0;
    for (uint32_t b = 0; b < K; ++b) T += (uint64_t)path_len(&mv[b]);
    if (T > step_cap) {
        bi->status = O_E_CAPACITY; bi->need_steps = (uint32_t)T; bi->need_batches = (uint32_t)T;
        return O_OK;
    }

    const uint32_t NONE = 0xFFFFFFFFu;
    size_t WH = (size_t)W * H;
    int rc = O_OK;
    ix_state X;
    memset(&X, 0, sizeof X);
    X.mv = mv; X.W = W; X.H = H;
    uint32_t *grp = (uint32_t *)malloc(sizeof(uint32_t) * K);
    X.len = (int *)malloc(sizeof(int) * K);
    X.pos = (int *)calloc(K, sizeof(int));
    X.rdir = (uint8_t *)calloc(K, 1);
    X.rx = (uint16_t *)calloc(K, sizeof(uint16_t));
    X.ry = (uint16_t *)calloc(K, sizeof(uint16_t));
    X.rowb = (sarr *)calloc((size_t)4 * H, sizeof(sarr));
    X.colb = (sarr *)calloc((size_t)4 * W, sizeof(sarr));
    uint32_t *last = (uint32_t *)malloc(sizeof(uint32_t) * WH);      /* last toucher of a trap */
    uint32_t *lastg = (uint32_t *)malloc(sizeof(uint32_t) * WH);     /* its group */
    uint32_t *seen = (uint32_t *)calloc(K, sizeof(uint32_t));
    uint32_t *gseen = (uint32_t *)calloc(G + 1, sizeof(uint32_t));
    int *indeg = (int *)calloc(K, sizeof(int));
    int *gwait = (int *)calloc(G + 1, sizeof(int));
    int *gremain = (int *)calloc(G + 1, sizeof(int));
    u32vec *succ = (u32vec *)calloc(K, sizeof(u32vec));
    u32vec *gsucc = (u32vec *)calloc(G + 1, sizeof(u32vec));
    uint32_t *stamp = (uint32_t *)calloc(WH, sizeof(uint32_t));
    uint32_t *acc = (uint32_t *)malloc(sizeof(uint32_t) * K);
    if (!grp || !X.len || !X.pos || !X.rdir || !X.rx || !X.ry || !X.rowb || !X.colb || !last || !lastg || !seen ||
        !gseen || !indeg || !gwait || !gremain || !succ || !gsucc || !stamp || !acc) { rc = O_E_NOMEM; goto done; }

    for (uint32_t g = 0; g < G; ++g)
        for (uint32_t b = goff[g]; b < goff[g + 1]; ++b) { grp[b] = g; gremain[g]++; }
    for (uint32_t b = 0; b < K; ++b) X.len[b] = path_len(&mv[b]);
    for (size_t c = 0; c < WH; ++c) { last[c] = NONE; lastg[c] = NONE; }

    /* reduced Gamma, groups and moves in order */
    for (uint32_t g = 0; g < G; ++g)
        for (uint32_t b = goff[g]; b < goff[g + 1]; ++b)
            for (int s = 0; s <= X.len[b]; ++s) {
                int x, y; path_cell(&mv[b], s, &x, &y);
                size_t c = (size_t)y * W + x;
                uint32_t pg = lastg[c];
                if (pg == g) {
                    uint32_t a = last[c];
                    if (seen[a] != b + 1) { seen[a] = b + 1; uv_push(&succ[a], b); indeg[b]++; }
                } else if (pg != NONE && gseen[pg] != g + 1) {
                    gseen[pg] = g + 1; uv_push(&gsucc[pg], g); gwait[g]++;
                }
                last[c] = b; lastg[c] = g;
            }
    for (uint32_t b = 0; b < K; ++b) if (succ[b].oom) { rc = O_E_NOMEM; goto done; }
    for (uint32_t g = 0; g < G; ++g) if (gsucc[g].oom) { rc = O_E_NOMEM; goto done; }

    for (uint32_t b = 0; b < K; ++b)
        if (indeg[b] == 0 && gwait[grp[b]] == 0) ix_make_ready(&X, b);

    uint64_t n_alive = K, n_out = 0, nb = 0;
    uint32_t iter = 0;
    if (batch_off) batch_off[0] = 0;
    while (n_alive > 0 && !X.oom) {
        if (X.ready.n == 0) { bi->status = O_E_INTERNAL; goto done; }
        ++iter;
        uint32_t na = 0;
        o_step e;
        /* the first move of Q always joins */
        uint32_t lead = X.ready.a[0];
        o_step L;
        ix_step(&X, lead, &L);
        acc[na++] = lead;
        stamp[(size_t)L.uy * W + L.ux] = iter;
        stamp[(size_t)L.vy * W + L.vx] = iter;
        if (flags == O_LAMBDA_NONE) {
            for (uint32_t q = 1; q < X.ready.n; ++q) {
                uint32_t b = X.ready.a[q];
                ix_step(&X, b, &e);
                if (stamp[(size_t)e.uy * W + e.ux] == iter || stamp[(size_t)e.vy * W + e.vx] == iter) continue;
                acc[na++] = b;
                stamp[(size_t)e.uy * W + e.ux] = iter;
                stamp[(size_t)e.vy * W + e.vx] = iter;
            }
        } else {
            const sarr *rb = &X.rowb[L.dir * H + L.uy], *cb = &X.colb[L.dir * W + L.ux];
            int use_row = 1, use_col = 1;
            if (flags == O_LAMBDA_ALONG) { if (L.dir >= 2) use_row = 0; else use_col = 0; }
            uint32_t ir = 0, ic = 0;
            for (;;) {
                uint32_t br = (use_row && ir < rb->n) ? rb->a[ir] : NONE;
                uint32_t bc = (use_col && ic < cb->n) ? cb->a[ic] : NONE;
                if (br == NONE && bc == NONE) break;
                int from_row = br < bc;
                uint32_t b = from_row ? br : bc;
                if (from_row) ir++; else ic++;
                if (b == lead) continue;
                ix_step(&X, b, &e);
                if (stamp[(size_t)e.uy * W + e.ux] == iter || stamp[(size_t)e.vy * W + e.vx] == iter) continue;
                acc[na++] = b;
                stamp[(size_t)e.uy * W + e.ux] = iter;
                stamp[(size_t)e.vy * W + e.vx] = iter;
                if (flags == O_LAMBDA_LINE_OR_COL && na == 2) {      /* the line is fixed */
                    if (from_row) use_col = 0; else use_row = 0;
                }
            }
        }
        /* emit the batch in acceptance order, then advance, finish and release */
        for (uint32_t k = 0; k < na; ++k) {
            ix_step(&X, acc[k], &e);
            if (steps) steps[n_out] = ((uint32_t)e.dir << 30) | ((uint32_t)e.ux << 15) | (uint32_t)e.uy;
            n_out++;
        }
        ++nb;
        if (batch_off && nb <= batch_cap) batch_off[nb] = (uint32_t)n_out;
        for (uint32_t k = 0; k < na; ++k) {
            uint32_t b = acc[k];
            ix_unready(&X, b);
            X.pos[b]++;
            if (X.pos[b] < X.len[b]) { ix_make_ready(&X, b); continue; }
            n_alive--;
            for (size_t s = 0; s < succ[b].n; ++s) {
                uint32_t t = succ[b].a[s];
                if (--indeg[t] == 0 && gwait[grp[t]] == 0) ix_make_ready(&X, t);
            }
            uint32_t g = grp[b];
            if (--gremain[g] == 0)
                for (size_t s = 0; s < gsucc[g].n; ++s) {
                    uint32_t h = gsucc[g].a[s];
                    if (--gwait[h] == 0)
                        for (uint32_t m = goff[h]; m < goff[h + 1]; ++m)
                            if (indeg[m] == 0 && X.pos[m] < X.len[m]) ix_make_ready(&X, m);
                }
        }
    }
    if (X.oom) { rc = O_E_NOMEM; goto done; }
    bi->need_batches = (uint32_t)nb;
    bi->need_steps = (uint32_t)n_out;
    if (nb > batch_cap || !batch_off || (n_out && !steps)) { bi->status = O_E_CAPACITY; goto done; }
    bi->status = O_OK;
    bi->n_batches = (uint32_t)nb;
    bi->n_steps = (uint32_t)n_out;
done:
    if (succ) for (uint32_t b = 0; b < K; ++b) free(succ[b].a);
    if (gsucc) for (uint32_t g = 0; g <= G; ++g) free(gsucc[g].a);
    if (X.rowb) for (int k = 0; k < 4 * H; ++k) free(X.rowb[k].a);
    if (X.colb) for (int k = 0; k < 4 * W; ++k) free(X.colb[k].a);
    free(X.ready.a);
    free(grp); free(X.len); free(X.pos); free(X.rdir); free(X.rx); free(X.ry); free(X.rowb); free(X.colb);
    free(last); free(lastg); free(seen); free(gseen); free(indeg); free(gwait); free(gremain); free(succ);
    free(gsucc); free(stamp); free(acc);
    return rc;
}
