/*
 * CPU oracle for the sparse-grid hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code with the HIP path: its data structure
 * (a root table of int32 slot indices over a growable pool of 8^3 blocks) and
 * every loop here are written independently, straight from the paper's
 * definitions, single-threaded and in program order.
 *
 * Semantics followed (paper, Section 3 "Spatially sparse programming" and
 * Section 4 "States"):
 *   - the domain is a root of R^3 cells over dense 8^3 leaf blocks; a block is
 *     active or not as a whole (dense leaves are all-or-nothing, Fig. 3);
 *   - every voxel has a value; an inactive voxel (and, by our reading, a voxel
 *     outside the domain) reads as the ambient value 0;
 *   - activation on write: activating an inactive block zero-fills it;
 *     activating an active block changes nothing;
 *   - list generation: the list of active root cells, consumed by struct-fors.
 *     The oracle emits it in ascending linear root index;
 *   - a struct-for visits every voxel of every listed block.
 *
 * Arithmetic is done in REAL (float or double, chosen at compile time) in the
 * exact operation order documented on each function, built with
 * -ffp-contract=off so no fused multiply-add changes the rounding.
 * Particle-to-grid transfer accumulates in double regardless of REAL and can
 * also return, per node and channel, the sum of absolute terms (the bound a
 * summation-order error is measured against).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef REAL
#define REAL float
#endif

#define BS 8
#define BV 512

typedef struct {
    int n;            /* domain edge in voxels */
    int R;            /* root edge in blocks */
    int channels;
    int64_t ncells;   /* R^3 */
    int32_t *root;    /* slot of each root cell, -1 when inactive */
    int64_t nslots;   /* slots in use */
    int64_t capslots; /* slots allocated */
    REAL **pool;      /* per channel: capslots * 512 values */
    int32_t *list;    /* list state: active root cells */
    int64_t count;    /* list length */
} og_grid;

/* ------------------------------------------------------------------ grid */

og_grid *og_create(int n, int channels) {
    if (n <= 0 || n % BS != 0 || channels <= 0) return NULL;
    og_grid *g = (og_grid *)calloc(1, sizeof(og_grid));
    g->n = n;
    g->R = n / BS;
    g->channels = channels;
    g->ncells = (int64_t)g->R * g->R * g->R;
    g->root = (int32_t *)malloc(sizeof(int32_t) * g->ncells);
    for (int64_t c = 0; c < g->ncells; ++c) g->root[c] = -1;
    g->list = (int32_t *)malloc(sizeof(int32_t) * g->ncells);
    g->count = 0;
    g->capslots = 16;
    g->nslots = 0;
    g->pool = (REAL **)calloc(channels, sizeof(REAL *));
    for (int ch = 0; ch < channels; ++ch)
        g->pool[ch] = (REAL *)calloc((size_t)g->capslots * BV, sizeof(REAL));
    return g;
}

void og_destroy(og_grid *g) {
    if (!g) return;
    for (int ch = 0; ch < g->channels; ++ch) free(g->pool[ch]);
    free(g->pool);
    free(g->root);
    free(g->list);
    free(g);
}

int og_root_edge(const og_grid *g) { return g->R; }
int64_t og_num_slots(const og_grid *g) { return g->nslots; }

static int64_t cell_of_block(const og_grid *g, int bi, int bj, int bk) {
    return ((int64_t)bi * g->R + bj) * g->R + bk;
}

static int block_in_domain(const og_grid *g, int bi, int bj, int bk) {
    return bi >= 0 && bj >= 0 && bk >= 0 && bi < g->R && bj < g->R && bk < g->R;
}

/* Activate one block: if it is inactive, give it a fresh slot and zero every
 * channel of that slot; otherwise nothing happens. */
static void activate_block(og_grid *g, int bi, int bj, int bk) {
    int64_t c = cell_of_block(g, bi, bj, bk);
    if (g->root[c] >= 0) return;
    if (g->nslots == g->capslots) {
        int64_t ncap = g->capslots * 2;
        for (int ch = 0; ch < g->channels; ++ch) {
            g->pool[ch] = (REAL *)realloc(g->pool[ch], sizeof(REAL) * (size_t)ncap * BV);
        }
        g->capslots = ncap;
    }
    int64_t s = g->nslots++;
    for (int ch = 0; ch < g->channels; ++ch)
        for (int v = 0; v < BV; ++v) g->pool[ch][s * BV + v] = (REAL)0;
    g->root[c] = (int32_t)s;
}

int og_is_active(const og_grid *g, int bi, int bj, int bk) {
    if (!block_in_domain(g, bi, bj, bk)) return 0;
    return g->root[cell_of_block(g, bi, bj, bk)] >= 0;
}

/* Activate coordinates in the given order.  coord_kind 0: voxel (i, j, k),
 * whose block is activated; 1: block (bi, bj, bk).  Returns the number of
 * coordinates that fell outside the domain (those are ignored). */
int64_t og_activate(og_grid *g, const int32_t *ijk, int64_t n, int coord_kind) {
    int64_t bad = 0;
    for (int64_t t = 0; t < n; ++t) {
        int a = ijk[3 * t], b = ijk[3 * t + 1], c = ijk[3 * t + 2];
        if (coord_kind == 0) {
            if (a < 0 || b < 0 || c < 0 || a >= g->n || b >= g->n || c >= g->n) { ++bad; continue; }
            a /= BS; b /= BS; c /= BS;
        } else if (!block_in_domain(g, a, b, c)) { ++bad; continue; }
        activate_block(g, a, b, c);
    }
    return bad;
}

/* List generation: every active root cell, ascending linear index. */
int64_t og_listgen(og_grid *g) {
    int64_t cnt = 0;
    for (int64_t c = 0; c < g->ncells; ++c)
        if (g->root[c] >= 0) g->list[cnt++] = (int32_t)c;
    g->count = cnt;
    return cnt;
}

/* Active root cells read from the mask (ascending), without touching the
 * list state. */
int64_t og_active_cells(const og_grid *g, int32_t *out) {
    int64_t cnt = 0;
    for (int64_t c = 0; c < g->ncells; ++c)
        if (g->root[c] >= 0) out[cnt++] = (int32_t)c;
    return cnt;
}

/* Replace the list state (test helper: lets a test run a struct-for over a
 * chosen subset of blocks, e.g. one block at a time). */
void og_set_list(og_grid *g, const int32_t *cells, int64_t n) {
    memcpy(g->list, cells, sizeof(int32_t) * (size_t)n);
    g->count = n;
}

int64_t og_get_list(const og_grid *g, int32_t *out) {
    memcpy(out, g->list, sizeof(int32_t) * (size_t)g->count);
    return g->count;
}

/* Value read with sparse semantics: 0 outside the domain or in an inactive
 * block. */
static REAL rd(const og_grid *g, int ch, int i, int j, int k) {
    if (i < 0 || j < 0 || k < 0 || i >= g->n || j >= g->n || k >= g->n) return (REAL)0;
    int32_t s = g->root[cell_of_block(g, i / BS, j / BS, k / BS)];
    if (s < 0) return (REAL)0;
    return g->pool[ch][(int64_t)s * BV + (i % BS) * 64 + (j % BS) * 8 + (k % BS)];
}

/* Activating write (activation on write). */
static void wr(og_grid *g, int ch, int i, int j, int k, REAL v) {
    activate_block(g, i / BS, j / BS, k / BS);
    int32_t s = g->root[cell_of_block(g, i / BS, j / BS, k / BS)];
    g->pool[ch][(int64_t)s * BV + (i % BS) * 64 + (j % BS) * 8 + (k % BS)] = v;
}

REAL og_read(const og_grid *g, int ch, int i, int j, int k) { return rd(g, ch, i, j, k); }

/* Copy the 512 values of root cell `cell` (zeros if inactive). */
void og_read_block(const og_grid *g, int ch, int32_t cell, REAL *out) {
    int32_t s = (cell >= 0 && cell < g->ncells) ? g->root[cell] : -1;
    for (int v = 0; v < BV; ++v) out[v] = s < 0 ? (REAL)0 : g->pool[ch][(int64_t)s * BV + v];
}

/* Store 512 values into root cell `cell`, activating it first. */
void og_write_block(og_grid *g, int ch, int32_t cell, const REAL *vals) {
    int bi = (int)(cell / ((int64_t)g->R * g->R)), bj = (int)((cell / g->R) % g->R), bk = (int)(cell % g->R);
    activate_block(g, bi, bj, bk);
    int32_t s = g->root[cell];
    for (int v = 0; v < BV; ++v) g->pool[ch][(int64_t)s * BV + v] = vals[v];
}

/* ------------------------------------------------ struct-for over the list */

/* Voxel coordinates of local voxel v of listed root cell `cell`. */
#define FOR_EACH_LISTED_VOXEL(g, ...)                                               \
    for (int64_t e = 0; e < (g)->count; ++e) {                                      \
        int64_t cell_ = (g)->list[e];                                               \
        int bi_ = (int)(cell_ / ((int64_t)(g)->R * (g)->R));                        \
        int bj_ = (int)((cell_ / (g)->R) % (g)->R);                                 \
        int bk_ = (int)(cell_ % (g)->R);                                            \
        for (int li = 0; li < BS; ++li)                                             \
            for (int lj = 0; lj < BS; ++lj)                                         \
                for (int lk = 0; lk < BS; ++lk) {                                   \
                    int i = bi_ * BS + li, j = bj_ * BS + lj, k = bk_ * BS + lk;    \
                    __VA_ARGS__                                                     \
                }                                                                   \
    }

/* Semi-Lagrangian advection, the building block of the MacCormack benchmark
 * (Section 8.2) and of the supplement's simple advection microbenchmark:
 * every listed voxel I takes q at the back-traced point p = I - dt * v(I)
 * (grid units, one Euler step; v in channels ch_v .. ch_v + 2), trilinearly
 * interpolated from the 8 voxels around p (or the RK3 back-trace below).
 * Reads outside the domain or in inactive blocks give 0.  Fixed order: corners (a, b, c) in {0, 1}^3
 * lexicographic, weight (wx[a] * wy[b]) * wz[c], s = s + w * q.  A point
 * further than 2 voxels outside the domain is moved to 2 voxels outside (all
 * its corners read 0 either way), which keeps the corner indices in range. */
static REAL clamp_coord(REAL p, int n) {
    if (p < (REAL)-2) return (REAL)-2;
    if (p > (REAL)(n + 1)) return (REAL)(n + 1);
    return p;
}

/* Trilinear sample of channel ch at point p (sparse reads, fixed corner order,
 * weight (wx * wy) * wz, s = s + w * q).  p is clamped as described above. */
static REAL sample_at(const og_grid *g, int ch, const REAL p_in[3]) {
    int base[3];
    REAL w[3][2];
    for (int d = 0; d < 3; ++d) {
        REAL p = clamp_coord(p_in[d], g->n);
        REAL b = (REAL)floor((double)p);
        REAL f = p - b;
        base[d] = (int)b;
        w[d][0] = (REAL)1 - f;
        w[d][1] = f;
    }
    REAL s = (REAL)0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
                REAL wt = (w[0][a] * w[1][b]) * w[2][c];
                s = s + wt * rd(g, ch, base[0] + a, base[1] + b, base[2] + c);
            }
    return s;
}

/* Back-traced point of voxel (i, j, k) over dt: one Euler step
 * p = I - dt * v(I), or (rk3) the three-stage Runge-Kutta back-trace
 *   v1 = v(I), p1 = I - (0.5 dt) v1, v2 = v(p1), p2 = I - (0.75 dt) v2,
 *   v3 = v(p2), p = I - dt * (2/9 v1 + 1/3 v2 + 4/9 v3)
 * with v sampled trilinearly; per component in that order. */
static void backtrace(const og_grid *g, int ch_v, int i, int j, int k, REAL dt, int rk3, REAL p[3]) {
    const REAL I[3] = {(REAL)i, (REAL)j, (REAL)k};
    REAL v1[3];
    for (int d = 0; d < 3; ++d) v1[d] = rd(g, ch_v + d, i, j, k);
    if (!rk3) {
        for (int d = 0; d < 3; ++d) p[d] = I[d] - dt * v1[d];
        return;
    }
    const REAL h1 = (REAL)0.5 * dt, h2 = (REAL)0.75 * dt;
    REAL p1[3], v2[3], p2[3], v3[3];
    for (int d = 0; d < 3; ++d) p1[d] = I[d] - h1 * v1[d];
    for (int d = 0; d < 3; ++d) v2[d] = sample_at(g, ch_v + d, p1);
    for (int d = 0; d < 3; ++d) p2[d] = I[d] - h2 * v2[d];
    for (int d = 0; d < 3; ++d) v3[d] = sample_at(g, ch_v + d, p2);
    const REAL c1 = (REAL)(2.0 / 9.0), c2 = (REAL)(1.0 / 3.0), c3 = (REAL)(4.0 / 9.0);
    for (int d = 0; d < 3; ++d) {
        REAL sv = c1 * v1[d];
        sv = sv + c2 * v2[d];
        sv = sv + c3 * v3[d];
        p[d] = I[d] - dt * sv;
    }
}

void og_advect_sl(og_grid *g, int ch_q, int ch_v, int ch_out, REAL dt, int rk3) {
    FOR_EACH_LISTED_VOXEL(g, {
        REAL p[3];
        backtrace(g, ch_v, i, j, k, dt, rk3, p);
        wr(g, ch_out, i, j, k, sample_at(g, ch_q, p));
    })
}

/* MacCormack correction with clamping (Section 8.2, after Selle et al.'s
 * unconditionally stable MacCormack method): given the forward
 * semi-Lagrangian result fwd = SL(q, v, dt) and the backward one
 * bwd = SL(fwd, v, -dt), every listed voxel I gets
 *   val = fwd[I] + 0.5 * (q[I] - bwd[I]),
 * clamped to the range of q over the 8 corners around the forward
 * back-traced point I - dt * v(I) (corner reads with sparse semantics; the
 * same clamping of far points as og_advect_sl).  Order: d = q - bwd,
 * h = 0.5 * d, val = fwd + h; min and max in corner order. */
void og_maccormack(og_grid *g, int ch_q, int ch_v, int ch_fwd, int ch_bwd, int ch_out, REAL dt, int rk3) {
    FOR_EACH_LISTED_VOXEL(g, {
        REAL p[3];
        backtrace(g, ch_v, i, j, k, dt, rk3, p);
        int base[3];
        for (int d = 0; d < 3; ++d) base[d] = (int)floor((double)clamp_coord(p[d], g->n));
        REAL lo = (REAL)0, hi = (REAL)0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) {
                    REAL x = rd(g, ch_q, base[0] + a, base[1] + b, base[2] + c);
                    if (a + b + c == 0) { lo = x; hi = x; }
                    else { lo = x < lo ? x : lo; hi = x > hi ? x : hi; }
                }
        REAL d = rd(g, ch_q, i, j, k) - rd(g, ch_bwd, i, j, k);
        REAL h = (REAL)0.5 * d;
        REAL val = rd(g, ch_fwd, i, j, k) + h;
        wr(g, ch_out, i, j, k, val < lo ? lo : (val > hi ? hi : val));
    })
}

/* ------------------------------------------ two-level transfers (Sec. 6.3)
 * A coarse grid has half the fine domain edge; fine voxel (i, j, k) lies
 * under coarse voxel (i/2, j/2, k/2).  Both transfers are struct-fors over
 * the FINE grid's list. */

/* Restriction (the downsample pattern of Section 6.3, in 3D): for every
 * listed fine voxel, in list order and ascending voxel order inside a block,
 * y[i/2, j/2, k/2] = y + w * x[i, j, k], writing the coarse grid with
 * activation on write (a coarse block is zero-filled when it is first
 * activated). */
void og_restrict(const og_grid *fine, og_grid *coarse, int ch_x, int ch_y, REAL w) {
    FOR_EACH_LISTED_VOXEL(fine, {
        REAL y = rd(coarse, ch_y, i / 2, j / 2, k / 2);
        REAL t = w * rd(fine, ch_x, i, j, k);
        wr(coarse, ch_y, i / 2, j / 2, k / 2, y + t);
    })
}

/* Prolongation by injection: for every listed fine voxel,
 * x[i, j, k] = x + y[i/2, j/2, k/2] (an inactive coarse voxel reads 0; the
 * coarse grid is not written). */
void og_prolong(const og_grid *coarse, og_grid *fine, int ch_y, int ch_x) {
    FOR_EACH_LISTED_VOXEL(fine, {
        REAL x = rd(fine, ch_x, i, j, k);
        REAL y = rd(coarse, ch_y, i / 2, j / 2, k / 2);
        wr(fine, ch_x, i, j, k, x + y);
    })
}

/* Sum of the six face neighbours, in the fixed order
 * ((((x[i-1] + x[i+1]) + x[j-1]) + x[j+1]) + x[k-1]) + x[k+1]. */
static REAL nbsum(const og_grid *g, int ch, int i, int j, int k) {
    REAL s = rd(g, ch, i - 1, j, k) + rd(g, ch, i + 1, j, k);
    s = s + rd(g, ch, i, j - 1, k);
    s = s + rd(g, ch, i, j + 1, k);
    s = s + rd(g, ch, i, j, k - 1);
    s = s + rd(g, ch, i, j, k + 1);
    return s;
}

/* out = a + coef * (s - 6 a): explicit step of the 7-point Laplacian in grid
 * units (h = 1). */
void og_lap_update(og_grid *g, int ch_a, int ch_out, REAL coef) {
    FOR_EACH_LISTED_VOXEL(g, {
        REAL a = rd(g, ch_a, i, j, k);
        REAL s = nbsum(g, ch_a, i, j, k);
        REAL six_a = (REAL)6 * a;
        REAL d = s - six_a;
        REAL t = coef * d;
        wr(g, ch_out, i, j, k, a + t);
    })
}

/* y = y + alpha * x */
void og_axpy(og_grid *g, int ch_y, int ch_x, REAL alpha) {
    FOR_EACH_LISTED_VOXEL(g, {
        REAL y = rd(g, ch_y, i, j, k);
        REAL t = alpha * rd(g, ch_x, i, j, k);
        wr(g, ch_y, i, j, k, y + t);
    })
}

/* One Jacobi sweep for -lap(x) = b in grid units: xn = (s + b) * fp(1/6). */
void og_jacobi(og_grid *g, int ch_x, int ch_b, int ch_xn) {
    const REAL sixth = (REAL)(1.0 / 6.0);
    FOR_EACH_LISTED_VOXEL(g, {
        REAL s = nbsum(g, ch_x, i, j, k);
        REAL b = rd(g, ch_b, i, j, k);
        REAL t = s + b;
        wr(g, ch_xn, i, j, k, t * sixth);
    })
}

/* dst = src */
void og_copy(og_grid *g, int ch_dst, int ch_src) {
    FOR_EACH_LISTED_VOXEL(g, { wr(g, ch_dst, i, j, k, rd(g, ch_src, i, j, k)); })
}

/* x = value */
void og_fill(og_grid *g, int ch, REAL value) {
    FOR_EACH_LISTED_VOXEL(g, { wr(g, ch, i, j, k, value); })
}

/* x = x + value */
void og_inc(og_grid *g, int ch, REAL value) {
    FOR_EACH_LISTED_VOXEL(g, { wr(g, ch, i, j, k, rd(g, ch, i, j, k) + value); })
}

/* Explicit diffusion step with face conductance kf = (k + k_nb) / 2:
 *   f = sum over faces (fixed order) of kf * (a_nb - a);  out = a + dt * f.
 * Reads of inactive neighbours (a_nb, k_nb) give 0. */
void og_diffuse(og_grid *g, int ch_a, int ch_k, int ch_out, REAL dt) {
    static const int off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    FOR_EACH_LISTED_VOXEL(g, {
        REAL a = rd(g, ch_a, i, j, k);
        REAL kc = rd(g, ch_k, i, j, k);
        REAL f = (REAL)0;
        for (int q = 0; q < 6; ++q) {
            int ii = i + off[q][0], jj = j + off[q][1], kk = k + off[q][2];
            REAL kf = (REAL)0.5 * (kc + rd(g, ch_k, ii, jj, kk));
            f = f + kf * (rd(g, ch_a, ii, jj, kk) - a);
        }
        wr(g, ch_out, i, j, k, a + dt * f);
    })
}

/* Reverse-mode step of og_diffuse.  With lam' the adjoint of the step's
 * output and a, k its inputs:
 *   lam[i]  = lam'[i] + dt * sum_faces kf * (lam'[nb] - lam'[i])
 *   gk[i]  += (dt * 0.5) * sum_faces (a[nb] - a[i]) * (lam'[i] - lam'[nb])
 * (the operator is self-adjoint; inactive neighbours read 0). */
void og_diffuse_adj(og_grid *g, int ch_a, int ch_k, int ch_lamn, int ch_lam, int ch_gk, REAL dt) {
    static const int off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    FOR_EACH_LISTED_VOXEL(g, {
        REAL l = rd(g, ch_lamn, i, j, k);
        REAL a = rd(g, ch_a, i, j, k);
        REAL kc = rd(g, ch_k, i, j, k);
        REAL f = (REAL)0, q2 = (REAL)0;
        for (int q = 0; q < 6; ++q) {
            int ii = i + off[q][0], jj = j + off[q][1], kk = k + off[q][2];
            REAL ln = rd(g, ch_lamn, ii, jj, kk);
            REAL kf = (REAL)0.5 * (kc + rd(g, ch_k, ii, jj, kk));
            f = f + kf * (ln - l);
            q2 = q2 + (rd(g, ch_a, ii, jj, kk) - a) * (l - ln);
        }
        wr(g, ch_lam, i, j, k, l + dt * f);
        REAL gk = rd(g, ch_gk, i, j, k);
        wr(g, ch_gk, i, j, k, gk + (dt * (REAL)0.5) * q2);
    })
}

/* ----------------------------------------------------------- particles */

/* x += dt * v, component by component (SoA: x[c*np + p]). */
void og_advect(REAL *x, const REAL *v, int64_t np, REAL dt) {
    for (int c = 0; c < 3; ++c)
        for (int64_t p = 0; p < np; ++p) x[c * np + p] = x[c * np + p] + dt * v[c * np + p];
}

/* Quadratic B-spline weights of one axis: base = floor(X - 1/2),
 * fx = X - base, w = (0.5 (1.5 - fx)^2, 0.75 - (fx - 1)^2, 0.5 (fx - 0.5)^2). */
static int bspline(REAL X, REAL w[3]) {
    int base = (int)floor((double)(X - (REAL)0.5));
    REAL fx = X - (REAL)base;
    REAL t0 = (REAL)1.5 - fx, t1 = fx - (REAL)1, t2 = fx - (REAL)0.5;
    w[0] = (REAL)0.5 * (t0 * t0);
    w[1] = (REAL)0.75 - t1 * t1;
    w[2] = (REAL)0.5 * (t2 * t2);
    return base;
}

/* Particle-to-grid transfer of mass and momentum (PIC), particles in id
 * order, the 27 nodes of each in (x, y, z) lexicographic order.  Each node's
 * block is activated on write.  Node weight w = (wx * wy) * wz; terms
 * w * m_p and (w * m_p) * v_p are formed in REAL and summed in double onto the current grid
 * values.  When ch_abs >= 0, channels ch_abs .. ch_abs+3 receive the sum of
 * |term| for m, mv0, mv1, mv2 (added to their current contents).
 * Returns the number of node writes that fell outside the domain (skipped). */
int64_t og_p2g(og_grid *g, int ch_m, int ch_mv, int ch_abs, const REAL *x, const REAL *v,
               const REAL *m, int64_t np, REAL inv_dx) {
    int64_t bad = 0;
    /* pass 1: activation, in exactly the order the writes happen */
    for (int64_t p = 0; p < np; ++p) {
        REAL w[3][3];
        int base[3];
        for (int c = 0; c < 3; ++c) base[c] = bspline(x[c * np + p] * inv_dx, w[c]);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int d = 0; d < 3; ++d) {
                    int i = base[0] + a, j = base[1] + b, k = base[2] + d;
                    if (i < 0 || j < 0 || k < 0 || i >= g->n || j >= g->n || k >= g->n) { ++bad; continue; }
                    activate_block(g, i / BS, j / BS, k / BS);
                }
    }
    /* pass 2: accumulate in double */
    int nacc = ch_abs >= 0 ? 8 : 4;
    size_t len = (size_t)g->nslots * BV;
    double *acc = (double *)malloc(sizeof(double) * len * nacc);
    for (int q = 0; q < 4; ++q) {
        int ch = q == 0 ? ch_m : ch_mv + q - 1;
        for (size_t t = 0; t < len; ++t) acc[q * len + t] = (double)g->pool[ch][t];
        if (ch_abs >= 0)
            for (size_t t = 0; t < len; ++t) acc[(4 + q) * len + t] = (double)g->pool[ch_abs + q][t];
    }
    for (int64_t p = 0; p < np; ++p) {
        REAL w[3][3];
        int base[3];
        for (int c = 0; c < 3; ++c) base[c] = bspline(x[c * np + p] * inv_dx, w[c]);
        REAL vp[3] = {v[p], v[np + p], v[2 * np + p]};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int d = 0; d < 3; ++d) {
                    int i = base[0] + a, j = base[1] + b, k = base[2] + d;
                    if (i < 0 || j < 0 || k < 0 || i >= g->n || j >= g->n || k >= g->n) continue;
                    int32_t s = g->root[cell_of_block(g, i / BS, j / BS, k / BS)];
                    size_t at = (size_t)s * BV + (i % BS) * 64 + (j % BS) * 8 + (k % BS);
                    REAL wt = (w[0][a] * w[1][b]) * w[2][d];
                    REAL term[4];
                    term[0] = wt * m[p];
                    for (int c = 0; c < 3; ++c) term[1 + c] = term[0] * vp[c];
                    for (int q = 0; q < 4; ++q) {
                        acc[q * len + at] += (double)term[q];
                        if (ch_abs >= 0) acc[(4 + q) * len + at] += fabs((double)term[q]);
                    }
                }
    }
    for (int q = 0; q < 4; ++q) {
        int ch = q == 0 ? ch_m : ch_mv + q - 1;
        for (size_t t = 0; t < len; ++t) g->pool[ch][t] = (REAL)acc[q * len + t];
        if (ch_abs >= 0)
            for (size_t t = 0; t < len; ++t) g->pool[ch_abs + q][t] = (REAL)acc[(4 + q) * len + t];
    }
    free(acc);
    return bad;
}

/* Grid velocity from momentum over the list: v = m > 0 ? mv / m : 0. */
void og_normalise(og_grid *g, int ch_m, int ch_mv, int ch_v) {
    FOR_EACH_LISTED_VOXEL(g, {
        REAL mm = rd(g, ch_m, i, j, k);
        for (int c = 0; c < 3; ++c) {
            REAL r = mm > (REAL)0 ? rd(g, ch_mv + c, i, j, k) / mm : (REAL)0;
            wr(g, ch_v + c, i, j, k, r);
        }
    })
}

/* Grid-to-particle gather of velocity: v_p = sum over the 27 nodes (same
 * order as og_p2g) of w * v_node, accumulated in REAL starting from 0. */
void og_g2p(const og_grid *g, int ch_v, const REAL *x, REAL *vout, int64_t np, REAL inv_dx) {
    for (int64_t p = 0; p < np; ++p) {
        REAL w[3][3];
        int base[3];
        for (int c = 0; c < 3; ++c) base[c] = bspline(x[c * np + p] * inv_dx, w[c]);
        REAL acc[3] = {(REAL)0, (REAL)0, (REAL)0};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int d = 0; d < 3; ++d) {
                    int i = base[0] + a, j = base[1] + b, k = base[2] + d;
                    REAL wt = (w[0][a] * w[1][b]) * w[2][d];
                    for (int c = 0; c < 3; ++c) acc[c] = acc[c] + wt * rd(g, ch_v + c, i, j, k);
                }
        for (int c = 0; c < 3; ++c) vout[c * np + p] = acc[c];
    }
}

/* B-spline weights of one coordinate, exposed for the pins. */
int og_bspline(REAL X, REAL *w3) { return bspline(X, w3); }

/* ------------------------------------------------------------- MLS-MPM
 * The particle-grid program of the paper's MLS-MPM benchmark (Section 8.3,
 * the falling cube of fixed-corotated particles), following the moving
 * least squares MPM it cites with APIC transfers: each particle carries a
 * position x, a velocity v, the affine velocity matrix C and the
 * deformation gradient F.  3x3 matrices are row-major, stored per particle
 * as SoA rows: M[(3 r + c) * np + p].  Node offsets and weights follow
 * og_p2g (quadratic B-spline, nodes in (x, y, z) lexicographic order); the
 * offset of node (a, b, d) from the particle in physical units is
 * dpos = ((a, b, d) - fx) * dx with fx = X - base per axis. */

static REAL det3(const REAL *A) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* Rotation R of the polar decomposition F = R S (S symmetric positive
 * definite), for det F > 0: Newton's iteration R <- (R + R^-T) / 2 from
 * R = F until no entry moves by more than a few units of rounding (at most
 * 100 iterations).  R^-T is the cofactor matrix over the determinant.
 * Returns the iterations taken, or -1 when det F <= 0. */
int og_polar(const REAL *F, REAL *R) {
    REAL X[9];
    for (int q = 0; q < 9; ++q) X[q] = F[q];
    if (!(det3(X) > (REAL)0)) return -1;
    const REAL tol = sizeof(REAL) == 8 ? (REAL)1e-15 : (REAL)2e-7;
    for (int it = 1; it <= 100; ++it) {
        REAL d = det3(X);
        REAL cof[9];
        cof[0] = X[4] * X[8] - X[5] * X[7];
        cof[1] = X[5] * X[6] - X[3] * X[8];
        cof[2] = X[3] * X[7] - X[4] * X[6];
        cof[3] = X[2] * X[7] - X[1] * X[8];
        cof[4] = X[0] * X[8] - X[2] * X[6];
        cof[5] = X[1] * X[6] - X[0] * X[7];
        cof[6] = X[1] * X[5] - X[2] * X[4];
        cof[7] = X[2] * X[3] - X[0] * X[5];
        cof[8] = X[0] * X[4] - X[1] * X[3];
        REAL moved = 0;
        for (int q = 0; q < 9; ++q) {
            REAL nx = (REAL)0.5 * (X[q] + cof[q] / d);
            REAL step = (REAL)fabs((double)(nx - X[q]));
            if (step > moved) moved = step;
            X[q] = nx;
        }
        if (moved <= tol) {
            for (int q = 0; q < 9; ++q) R[q] = X[q];
            return it;
        }
    }
    for (int q = 0; q < 9; ++q) R[q] = X[q];
    return 100;
}

/* Kirchhoff stress of the fixed-corotated model at F:
 * tau = 2 mu (F - R) F^T + lambda (J - 1) J I, J = det F, R from og_polar. */
void og_fcr_stress(const REAL *F, REAL mu, REAL lam, REAL *tau) {
    REAL R[9];
    og_polar(F, R);
    REAL J = det3(F);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            REAL s = 0;
            for (int k = 0; k < 3; ++k) s = s + (F[3 * r + k] - R[3 * r + k]) * F[3 * c + k];
            tau[3 * r + c] = (REAL)2 * mu * s + (r == c ? lam * (J - (REAL)1) * J : (REAL)0);
        }
}

/* MLS-MPM particle-to-grid transfer, particles in id order.  Per particle:
 *   F <- (I + dt C) F                          (stored back into F)
 *   A  = -(dt * vol * 4 * inv_dx^2) tau(F) + mass * C
 *   node (a, b, d) receives  m  += w * mass
 *                            mv += w * (mass * v + A dpos)
 * with w and dpos as above.  Activation and accumulation in double as in
 * og_p2g.  With ch_abs >= 0, channels ch_abs .. ch_abs + 3 receive the
 * error scale of each node's sum: the sum over its terms of the magnitudes
 * of the products each term is made of -- |w mass| for m and, for mv_c,
 * |w| (|mass v_c| + sum_e |A_ce|' |dpos_e|), where |A_ce|' bounds the
 * magnitudes inside A_ce: dt vol 4 inv_dx^2 (2 mu sum_k (|F_ck| + |R_ck|)
 * |F_ek| + |lambda (J - 1) J|) + mass |C_ce| (the difference F - R cancels,
 * so its rounding error is set by |F| and |R|, not by F - R).  Returns the
 * number of node writes outside the domain (skipped). */
int64_t og_mpm_p2g(og_grid *g, int ch_m, int ch_mv, int ch_abs, const REAL *x, const REAL *v,
                   const REAL *C, REAL *F, int64_t np, REAL inv_dx, REAL dt, REAL mass, REAL vol,
                   REAL mu, REAL lam) {
    int64_t bad = 0;
    for (int64_t p = 0; p < np; ++p) {
        REAL w[3][3];
        int base[3];
        for (int c = 0; c < 3; ++c) base[c] = bspline(x[c * np + p] * inv_dx, w[c]);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int d = 0; d < 3; ++d) {
                    int i = base[0] + a, j = base[1] + b, k = base[2] + d;
                    if (i < 0 || j < 0 || k < 0 || i >= g->n || j >= g->n || k >= g->n) { ++bad; continue; }
                    activate_block(g, i / BS, j / BS, k / BS);
                }
    }
    int nacc = ch_abs >= 0 ? 8 : 4;
    size_t len = (size_t)g->nslots * BV;
    double *acc = (double *)malloc(sizeof(double) * len * nacc);
    for (int q = 0; q < 4; ++q) {
        int ch = q == 0 ? ch_m : ch_mv + q - 1;
        for (size_t t = 0; t < len; ++t) acc[q * len + t] = (double)g->pool[ch][t];
        if (ch_abs >= 0)
            for (size_t t = 0; t < len; ++t) acc[(4 + q) * len + t] = (double)g->pool[ch_abs + q][t];
    }
    const REAL dx = (REAL)1 / inv_dx;
    const REAL kstress = dt * vol * (REAL)4 * inv_dx * inv_dx;
    for (int64_t p = 0; p < np; ++p) {
        REAL Cp[9], Fo[9], Fn[9], tau[9], A[9];
        for (int q = 0; q < 9; ++q) {
            Cp[q] = C[q * np + p];
            Fo[q] = F[q * np + p];
        }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                REAL s = 0;
                for (int k = 0; k < 3; ++k) s = s + ((r == k ? (REAL)1 : (REAL)0) + dt * Cp[3 * r + k]) * Fo[3 * k + c];
                Fn[3 * r + c] = s;
            }
        for (int q = 0; q < 9; ++q) F[q * np + p] = Fn[q];
        og_fcr_stress(Fn, mu, lam, tau);
        for (int q = 0; q < 9; ++q) A[q] = -(kstress * tau[q]) + mass * Cp[q];
        REAL Aabs[9];
        if (ch_abs >= 0) {
            REAL Rn[9];
            og_polar(Fn, Rn);
            REAL J = det3(Fn);
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    double sz = 0;
                    for (int k = 0; k < 3; ++k)
                        sz += (fabs((double)Fn[3 * r + k]) + fabs((double)Rn[3 * r + k])) * fabs((double)Fn[3 * c + k]);
                    double t = 2.0 * fabs((double)mu) * sz + (r == c ? fabs((double)(lam * (J - 1) * J)) : 0.0);
                    Aabs[3 * r + c] = (REAL)(fabs((double)kstress) * t + fabs((double)(mass * Cp[3 * r + c])));
                }
        }
        REAL w[3][3], fx[3];
        int base[3];
        for (int c = 0; c < 3; ++c) {
            REAL X = x[c * np + p] * inv_dx;
            base[c] = bspline(X, w[c]);
            fx[c] = X - (REAL)base[c];
        }
        REAL mvp[3] = {mass * v[p], mass * v[np + p], mass * v[2 * np + p]};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int d = 0; d < 3; ++d) {
                    int i = base[0] + a, j = base[1] + b, k = base[2] + d;
                    if (i < 0 || j < 0 || k < 0 || i >= g->n || j >= g->n || k >= g->n) continue;
                    int32_t s = g->root[cell_of_block(g, i / BS, j / BS, k / BS)];
                    size_t at = (size_t)s * BV + (i % BS) * 64 + (j % BS) * 8 + (k % BS);
                    REAL wt = (w[0][a] * w[1][b]) * w[2][d];
                    REAL dpos[3] = {((REAL)a - fx[0]) * dx, ((REAL)b - fx[1]) * dx, ((REAL)d - fx[2]) * dx};
                    REAL term[4];
                    term[0] = wt * mass;
                    for (int c = 0; c < 3; ++c) {
                        REAL ad = A[3 * c] * dpos[0] + A[3 * c + 1] * dpos[1] + A[3 * c + 2] * dpos[2];
                        term[1 + c] = wt * (mvp[c] + ad);
                    }
                    for (int q = 0; q < 4; ++q) acc[q * len + at] += (double)term[q];
                    if (ch_abs >= 0) {
                        acc[4 * len + at] += fabs((double)term[0]);
                        for (int c = 0; c < 3; ++c) {
                            double sz = fabs((double)mvp[c]);
                            for (int e = 0; e < 3; ++e) sz += fabs((double)Aabs[3 * c + e]) * fabs((double)dpos[e]);
                            acc[(5 + c) * len + at] += fabs((double)wt) * sz;
                        }
                    }
                }
    }
    for (int q = 0; q < 4; ++q) {
        REAL *dst = g->pool[q == 0 ? ch_m : ch_mv + q - 1];
        for (size_t t = 0; t < len; ++t) dst[t] = (REAL)acc[q * len + t];
        if (ch_abs >= 0)
            for (size_t t = 0; t < len; ++t) g->pool[ch_abs + q][t] = (REAL)acc[(4 + q) * len + t];
    }
    free(acc);
    return bad;
}

/* MLS-MPM grid update over the list: where m > 0, v = mv / m, then
 * v_z -= dt * gravity (z, axis 2, is up), then the walls: along each axis a
 * node within `bound` nodes of the low side (index < bound) loses a
 * negative velocity component and one beyond n - bound a positive one.
 * Where m == 0, v = 0. */
void og_mpm_grid(og_grid *g, int ch_m, int ch_mv, int ch_v, REAL dt, REAL gravity, int bound) {
    FOR_EACH_LISTED_VOXEL(g, {
        REAL mnode = rd(g, ch_m, i, j, k);
        REAL vv[3] = {(REAL)0, (REAL)0, (REAL)0};
        if (mnode > (REAL)0) {
            for (int c = 0; c < 3; ++c) vv[c] = rd(g, ch_mv + c, i, j, k) / mnode;
            vv[2] = vv[2] - dt * gravity;
            int idx[3] = {i, j, k};
            for (int c = 0; c < 3; ++c) {
                if (idx[c] < bound && vv[c] < (REAL)0) vv[c] = (REAL)0;
                if (idx[c] > g->n - bound && vv[c] > (REAL)0) vv[c] = (REAL)0;
            }
        }
        for (int c = 0; c < 3; ++c) wr(g, ch_v + c, i, j, k, vv[c]);
    })
}

/* MLS-MPM grid-to-particle gather: v_p = sum of w * v_node and
 * C_p = 4 inv_dx^2 * sum of w * v_node dpos^T over the 27 nodes, both
 * accumulated in REAL from 0 in node order (C as B_rc += (w * v_r) * dpos_c,
 * then scaled).  Nodes outside the domain or in inactive blocks read 0. */
void og_mpm_g2p(const og_grid *g, int ch_v, const REAL *x, REAL *vout, REAL *Cout, int64_t np, REAL inv_dx) {
    const REAL dx = (REAL)1 / inv_dx;
    const REAL kc = (REAL)4 * inv_dx * inv_dx;
    for (int64_t p = 0; p < np; ++p) {
        REAL w[3][3], fx[3];
        int base[3];
        for (int c = 0; c < 3; ++c) {
            REAL X = x[c * np + p] * inv_dx;
            base[c] = bspline(X, w[c]);
            fx[c] = X - (REAL)base[c];
        }
        REAL av[3] = {0, 0, 0}, B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int d = 0; d < 3; ++d) {
                    int i = base[0] + a, j = base[1] + b, k = base[2] + d;
                    REAL wt = (w[0][a] * w[1][b]) * w[2][d];
                    REAL off[3] = {((REAL)a - fx[0]) * dx, ((REAL)b - fx[1]) * dx, ((REAL)d - fx[2]) * dx};
                    for (int r = 0; r < 3; ++r) {
                        REAL wv = wt * rd(g, ch_v + r, i, j, k);
                        av[r] = av[r] + wv;
                        for (int c = 0; c < 3; ++c) B[3 * r + c] = B[3 * r + c] + wv * off[c];
                    }
                }
        for (int r = 0; r < 3; ++r) vout[r * np + p] = av[r];
        for (int q = 0; q < 9; ++q) Cout[q * np + p] = kc * B[q];
    }
}
