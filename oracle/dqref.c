/*
 * dqref.c - CPU oracle for SZ dual-quantisation (TEST INFRASTRUCTURE ONLY).
 *
 * Plain definitions, written for reading rather than speed: every element is
 * handled on its own, the Lorenzo residual is the full signed sum over the
 * 2^d corners of the unit cell, and decoding is the sequential
 * reconstruction the paper describes (Section III-A). OpenMP only spreads
 * whole blocks over threads; blocks are independent (Section III-F) and all
 * output ordering is fixed by sequential loops, so results do not depend on
 * the thread count.
 *
 * Readings of the paper that this file fixes (the paper's Algorithm 2
 * listing is not available, only its description in Section III-A):
 *  - prequantisation rounds the exact rational x / (2 eb) to the nearest
 *    integer, exact halves to even, and q must lie in [-(2^31-1), 2^31-1];
 *  - padding statistics are exact integer means of q, rounded half toward
 *    +infinity, or the minimum / maximum of q (block or global);
 *  - the edge padding of axis a is the mean of the block's own cells whose
 *    local coordinate along a is 0; a halo cell that lies in front of the
 *    block along several axes takes the rounded mean of those axes' values;
 *  - codes are uint16 with 0 reserved for outliers; outliers carry the
 *    residual delta; outliers are listed block by block, blocks in row-major
 *    order of the block grid, cells in local row-major order.
 */
#include "dqref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* largest accepted |q|: q must be an int32 with a representable negation */
static const int64_t QMAX = 2147483647; /* 2^31 - 1 */

typedef struct {
    int d;
    int64_t n[3];   /* extents, axis 0 slowest */
    int64_t nb[3];  /* blocks per axis */
    int64_t B;
    int64_t N;
    int64_t nblocks;
} geom;

static int popcount_u(unsigned v) {
    int c = 0;
    while (v) {
        c += (int)(v & 1u);
        v >>= 1;
    }
    return c;
}

int dqref_validate(const dqref_params *p) {
    if (!p) return DQREF_EINVAL;
    if (p->ndim < 1 || p->ndim > 3) return DQREF_EINVAL;
    double total = 1.0;
    for (int a = 0; a < p->ndim; ++a) {
        if (p->shape[a] < 1) return DQREF_EINVAL;
        total *= (double)p->shape[a];
    }
    if (total > 4294967295.0) return DQREF_EINVAL; /* indices are uint32 */
    if (!(p->eb > 0.0) || !isfinite(p->eb)) return DQREF_EINVAL;
    if (p->eb_mode != DQREF_EB_ABS && p->eb_mode != DQREF_EB_REL) return DQREF_EINVAL;
    if (p->eb_mode == DQREF_EB_ABS && !isfinite(1.0 / (2.0 * p->eb))) return DQREF_EINVAL;
    if (p->block < 1) return DQREF_EINVAL;
    if (p->pad_mode < DQREF_PAD_ZERO || p->pad_mode > DQREF_PAD_GIVEN) return DQREF_EINVAL;
    if (p->radius < 1 || p->radius > 32768) return DQREF_EINVAL;
    return DQREF_OK;
}

static void make_geom(const dqref_params *p, geom *g) {
    g->d = p->ndim;
    g->B = p->block;
    g->N = 1;
    g->nblocks = 1;
    for (int a = 0; a < 3; ++a) {
        g->n[a] = 1;
        g->nb[a] = 1;
    }
    for (int a = 0; a < g->d; ++a) {
        g->n[a] = p->shape[a];
        g->nb[a] = (p->shape[a] + g->B - 1) / g->B;
        g->N *= g->n[a];
        g->nblocks *= g->nb[a];
    }
}

int64_t dqref_num_blocks(const dqref_params *p) {
    if (dqref_validate(p) != DQREF_OK) return -1;
    geom g;
    make_geom(p, &g);
    return g.nblocks;
}

int64_t dqref_pad_count(const dqref_params *p) {
    if (dqref_validate(p) != DQREF_OK) return -1;
    geom g;
    make_geom(p, &g);
    switch (p->pad_mode) {
    case DQREF_PAD_ZERO: return 0;
    case DQREF_PAD_GLOBAL_MEAN:
    case DQREF_PAD_GLOBAL_MIN:
    case DQREF_PAD_GLOBAL_MAX: return 1;
    case DQREF_PAD_BLOCK_MEAN:
    case DQREF_PAD_BLOCK_MIN:
    case DQREF_PAD_BLOCK_MAX:
    case DQREF_PAD_GIVEN: return g.nblocks;
    default: return g.nblocks * g.d;
    }
}

/* floor((2S + n) / (2n)), computed without overflow in 128-bit integers */
int64_t dqref_round_mean(int64_t S, int64_t n) {
    __int128 num = (__int128)2 * S + n;
    __int128 den = (__int128)2 * n;
    __int128 quo = num / den; /* C division truncates toward zero */
    if (num % den != 0 && ((num < 0) != (den < 0))) quo -= 1;
    return (int64_t)quo;
}

/* C-order linear index of coordinates c */
static int64_t ravel(const geom *g, const int64_t *c) {
    int64_t lin = 0;
    for (int a = 0; a < g->d; ++a) lin = lin * g->n[a] + c[a];
    return lin;
}

static void unravel(const geom *g, int64_t lin, int64_t *c) {
    for (int a = g->d - 1; a >= 0; --a) {
        c[a] = lin % g->n[a];
        lin /= g->n[a];
    }
}

static void block_coords(const geom *g, int64_t b, int64_t *bc) {
    for (int a = g->d - 1; a >= 0; --a) {
        bc[a] = b % g->nb[a];
        b /= g->nb[a];
    }
}

/* in-field extent of block bc along each axis */
static void block_extent(const geom *g, const int64_t *bc, int64_t *ext) {
    for (int a = 0; a < g->d; ++a) {
        int64_t lo = bc[a] * g->B;
        int64_t hi = lo + g->B;
        if (hi > g->n[a]) hi = g->n[a];
        ext[a] = hi - lo;
    }
}

/* local coordinates u of the k-th in-field cell of a block (local row-major) */
static void local_coords(const geom *g, const int64_t *ext, int64_t k, int64_t *u) {
    for (int a = g->d - 1; a >= 0; --a) {
        u[a] = k % ext[a];
        k /= ext[a];
    }
}

static int64_t block_cells(const geom *g, const int64_t *ext) {
    int64_t c = 1;
    for (int a = 0; a < g->d; ++a) c *= ext[a];
    return c;
}

/* ------------------------------------------------------------ eb and q */

int dqref_resolve_eb(const dqref_params *p, const float *x, double *eb_abs) {
    int st = dqref_validate(p);
    if (st != DQREF_OK) return st;
    geom g;
    make_geom(p, &g);
    if (p->eb_mode == DQREF_EB_ABS) {
        *eb_abs = p->eb;
        return DQREF_OK;
    }
    /* value-range relative bound (Section II-B): eb = rel * (max - min) */
    float mn = INFINITY, mx = -INFINITY;
    for (int64_t i = 0; i < g.N; ++i) {
        if (!isfinite(x[i])) return DQREF_ERANGE;
        if (x[i] < mn) mn = x[i];
        if (x[i] > mx) mx = x[i];
    }
    double eb = p->eb * ((double)mx - (double)mn);
    if (!(eb > 0.0) || !isfinite(eb) || !isfinite(1.0 / (2.0 * eb))) return DQREF_EINVAL;
    *eb_abs = eb;
    return DQREF_OK;
}

/* Nearest integer to the exact rational x / two_eb, halves to even.
 * x = mx 2^ex and two_eb = md 2^ed with integer mantissas, so the quotient is
 * (mx / md) 2^(ex - ed), evaluated with 128-bit integer division.
 * Returns 0 on success, -1 when x is not finite or |q| > QMAX. */
static int quantize_exact(float xf, double two_eb, int64_t *qout) {
    if (!isfinite(xf)) return -1;
    if (xf == 0.0f) {
        *qout = 0;
        return 0;
    }
    int ex, ed;
    double fx = frexp((double)xf, &ex); /* 0.5 <= |fx| < 1 */
    double fd = frexp(two_eb, &ed);
    int64_t mx = (int64_t)ldexp(fx, 24); /* exact: a float has 24 bits */
    int64_t md = (int64_t)ldexp(fd, 53); /* exact: a double has 53 bits */
    int s = (ex - 24) - (ed - 53);
    __int128 num = mx, den = md;
    if (s >= 0) {
        if (s > 62) return -1; /* |x / two_eb| >= 2^(s-30) > 2^32 */
        num *= (__int128)1 << s; /* exact: |num| < 2^86 */
    } else {
        if (-s > 70) { /* |x / two_eb| < 2^24 / 2^(52+70): rounds to 0 */
            *qout = 0;
            return 0;
        }
        den *= (__int128)1 << -s; /* exact: den < 2^123 */
    }
    __int128 quo = num / den; /* truncates toward zero */
    __int128 rem = num - quo * den;
    __int128 twice = rem < 0 ? -2 * rem : 2 * rem;
    int sign = num < 0 ? -1 : 1;
    if (twice > den || (twice == den && (quo & 1) != 0)) quo += sign;
    if (quo > QMAX || quo < -QMAX) return -1;
    *qout = (int64_t)quo;
    return 0;
}

/* Pre-quantisation (Section III-A): q = round(x / (2 eb)), which gives
 * |x - 2 eb q| <= eb. The quotient is the exact rational one (2 eb being the
 * fp64 number 2*eb); exact halves go to the even integer. */
int dqref_prequantize(const dqref_params *p, const float *x, double eb_abs, int32_t *q) {
    int st = dqref_validate(p);
    if (st != DQREF_OK) return st;
    geom g;
    make_geom(p, &g);
    const double two_eb = 2.0 * eb_abs;
    int bad = 0;
    for (int64_t i = 0; i < g.N; ++i) {
        int64_t v;
        if (quantize_exact(x[i], two_eb, &v) != 0) {
            bad = 1;
            q[i] = 0;
            continue;
        }
        q[i] = (int32_t)v;
    }
    return bad ? DQREF_ERANGE : DQREF_OK;
}

/* ------------------------------------------------------------ padding */

/* Padding values (Section IV-A: a statistic of the data - mean, minimum or
 * maximum; IV-B: one value globally, one per block, or one per block and
 * axis). */
int dqref_pad_values(const dqref_params *p, const int32_t *q, int32_t *pads) {
    int st = dqref_validate(p);
    if (st != DQREF_OK) return st;
    geom g;
    make_geom(p, &g);
    if (p->pad_mode == DQREF_PAD_ZERO || p->pad_mode == DQREF_PAD_GIVEN) return DQREF_OK;
    if (p->pad_mode == DQREF_PAD_GLOBAL_MEAN) {
        int64_t S = 0;
        for (int64_t i = 0; i < g.N; ++i) S += q[i];
        pads[0] = (int32_t)dqref_round_mean(S, g.N);
        return DQREF_OK;
    }
    if (p->pad_mode == DQREF_PAD_GLOBAL_MIN || p->pad_mode == DQREF_PAD_GLOBAL_MAX) {
        int32_t lo = q[0], hi = q[0];
        for (int64_t i = 1; i < g.N; ++i) {
            if (q[i] < lo) lo = q[i];
            if (q[i] > hi) hi = q[i];
        }
        pads[0] = p->pad_mode == DQREF_PAD_GLOBAL_MIN ? lo : hi;
        return DQREF_OK;
    }
    for (int64_t b = 0; b < g.nblocks; ++b) {
        int64_t bc[3], ext[3], u[3], c[3];
        block_coords(&g, b, bc);
        block_extent(&g, bc, ext);
        int64_t cells = block_cells(&g, ext);
        int64_t S = 0, face_sum[3] = {0, 0, 0}, face_cnt[3] = {0, 0, 0};
        int32_t lo = 0, hi = 0;
        for (int64_t k = 0; k < cells; ++k) {
            local_coords(&g, ext, k, u);
            for (int a = 0; a < g.d; ++a) c[a] = bc[a] * g.B + u[a];
            int32_t v = q[ravel(&g, c)];
            S += v;
            if (k == 0 || v < lo) lo = v;
            if (k == 0 || v > hi) hi = v;
            for (int a = 0; a < g.d; ++a) {
                if (u[a] == 0) {
                    face_sum[a] += v;
                    face_cnt[a] += 1;
                }
            }
        }
        if (p->pad_mode == DQREF_PAD_BLOCK_MEAN) {
            pads[b] = (int32_t)dqref_round_mean(S, cells);
        } else if (p->pad_mode == DQREF_PAD_BLOCK_MIN) {
            pads[b] = lo;
        } else if (p->pad_mode == DQREF_PAD_BLOCK_MAX) {
            pads[b] = hi;
        } else {
            for (int a = 0; a < g.d; ++a)
                pads[b * g.d + a] = (int32_t)dqref_round_mean(face_sum[a], face_cnt[a]);
        }
    }
    return DQREF_OK;
}

/* Value of a halo cell in front of block b. The cell lies at local
 * coordinate -1 along exactly the axes in the bit set H (H != 0). */
static int32_t halo_value(const dqref_params *p, const geom *g, const int32_t *pads,
                          int64_t b, unsigned H) {
    switch (p->pad_mode) {
    case DQREF_PAD_ZERO: return 0;
    case DQREF_PAD_GLOBAL_MEAN:
    case DQREF_PAD_GLOBAL_MIN:
    case DQREF_PAD_GLOBAL_MAX: return pads[0];
    case DQREF_PAD_BLOCK_MEAN:
    case DQREF_PAD_BLOCK_MIN:
    case DQREF_PAD_BLOCK_MAX:
    case DQREF_PAD_GIVEN: return pads[b];
    default: {
        int64_t S = 0;
        int m = popcount_u(H);
        for (int a = 0; a < g->d; ++a)
            if (H & (1u << a)) S += pads[b * g->d + a];
        if (m == 1) return (int32_t)S;
        return (int32_t)dqref_round_mean(S, m);
    }
    }
}

/* v(w): q at local coordinates w of block b (origin o), or the halo value
 * when some coordinate is -1. src holds q in natural layout. */
static uint32_t cell_value(const dqref_params *p, const geom *g, const int32_t *src,
                           const int32_t *pads, int64_t b, const int64_t *o,
                           const int64_t *w) {
    unsigned H = 0;
    for (int a = 0; a < g->d; ++a)
        if (w[a] < 0) H |= 1u << a;
    if (H) return (uint32_t)halo_value(p, g, pads, b, H);
    int64_t c[3];
    for (int a = 0; a < g->d; ++a) c[a] = o[a] + w[a];
    return (uint32_t)src[ravel(g, c)];
}

/* The non-central part of the Lorenzo stencil at local cell u:
 * sum over non-empty axis sets S of (-1)^|S| v(u - 1_S). The residual is
 * v(u) plus this sum; the prediction is minus this sum. */
static uint32_t lorenzo_neighbour_sum(const dqref_params *p, const geom *g,
                                      const int32_t *src, const int32_t *pads, int64_t b,
                                      const int64_t *o, const int64_t *u) {
    uint32_t acc = 0;
    for (unsigned S = 1; S < (1u << g->d); ++S) {
        int64_t w[3];
        for (int a = 0; a < g->d; ++a) w[a] = u[a] - (int64_t)((S >> a) & 1u);
        uint32_t v = cell_value(p, g, src, pads, b, o, w);
        if (popcount_u(S) & 1) acc -= v;
        else acc += v;
    }
    return acc;
}

/* ------------------------------------------------------------ residuals */

/* Post-quantisation input (Section III-A): delta = q - p with p the Lorenzo
 * prediction of q from its lower neighbours in the same block, the padding
 * standing in for neighbours outside the block. */
int dqref_residuals(const dqref_params *p, const int32_t *q, const int32_t *pads,
                    int32_t *delta, int nthreads) {
    int st = dqref_validate(p);
    if (st != DQREF_OK) return st;
    geom g;
    make_geom(p, &g);
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 64)
#endif
    for (int64_t b = 0; b < g.nblocks; ++b) {
        int64_t bc[3], ext[3], o[3], u[3], c[3];
        block_coords(&g, b, bc);
        block_extent(&g, bc, ext);
        for (int a = 0; a < g.d; ++a) o[a] = bc[a] * g.B;
        int64_t cells = block_cells(&g, ext);
        for (int64_t k = 0; k < cells; ++k) {
            local_coords(&g, ext, k, u);
            for (int a = 0; a < g.d; ++a) c[a] = o[a] + u[a];
            int64_t i = ravel(&g, c);
            uint32_t r = (uint32_t)q[i] + lorenzo_neighbour_sum(p, &g, q, pads, b, o, u);
            delta[i] = (int32_t)r;
        }
    }
    (void)nthreads;
    return DQREF_OK;
}

/* Decompression (Section III-A): each point is rebuilt after the points it
 * is predicted from, q(u) = delta(u) - sum_{S != 0} (-1)^|S| v(u - 1_S). */
int dqref_reconstruct(const dqref_params *p, const int32_t *delta, const int32_t *pads,
                      int32_t *q, int nthreads) {
    int st = dqref_validate(p);
    if (st != DQREF_OK) return st;
    geom g;
    make_geom(p, &g);
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 64)
#endif
    for (int64_t b = 0; b < g.nblocks; ++b) {
        int64_t bc[3], ext[3], o[3], u[3], c[3];
        block_coords(&g, b, bc);
        block_extent(&g, bc, ext);
        for (int a = 0; a < g.d; ++a) o[a] = bc[a] * g.B;
        int64_t cells = block_cells(&g, ext);
        for (int64_t k = 0; k < cells; ++k) { /* local row-major: neighbours first */
            local_coords(&g, ext, k, u);
            for (int a = 0; a < g.d; ++a) c[a] = o[a] + u[a];
            int64_t i = ravel(&g, c);
            uint32_t v = (uint32_t)delta[i] - lorenzo_neighbour_sum(p, &g, q, pads, b, o, u);
            q[i] = (int32_t)v;
        }
    }
    (void)nthreads;
    return DQREF_OK;
}

/* ------------------------------------------------------------ compress */

int dqref_compress(const dqref_params *p, const float *x, uint16_t *codes,
                   uint32_t *out_idx, int32_t *out_val, uint64_t out_cap,
                   uint64_t *n_out, int32_t *pads, double *eb_abs, int nthreads) {
    int st = dqref_validate(p);
    if (st != DQREF_OK) return st;
    geom g;
    make_geom(p, &g);
    *n_out = 0;
    double eb;
    st = dqref_resolve_eb(p, x, &eb);
    if (st != DQREF_OK) return st;
    *eb_abs = eb;
    int32_t *q = (int32_t *)malloc((size_t)g.N * sizeof(int32_t));
    int32_t *delta = (int32_t *)malloc((size_t)g.N * sizeof(int32_t));
    if (!q || !delta) {
        free(q);
        free(delta);
        return DQREF_EINVAL;
    }
    st = dqref_prequantize(p, x, eb, q);
    if (st == DQREF_OK) st = dqref_pad_values(p, q, pads);
    if (st == DQREF_OK) st = dqref_residuals(p, q, pads, delta, nthreads);
    if (st == DQREF_OK) {
        /* Post-quantisation to codes; outliers emitted block by block. */
        const int64_t R = p->radius;
        uint64_t cnt = 0;
        for (int64_t b = 0; b < g.nblocks; ++b) {
            int64_t bc[3], ext[3], u[3], c[3];
            block_coords(&g, b, bc);
            block_extent(&g, bc, ext);
            int64_t cells = block_cells(&g, ext);
            for (int64_t k = 0; k < cells; ++k) {
                local_coords(&g, ext, k, u);
                for (int a = 0; a < g.d; ++a) c[a] = bc[a] * g.B + u[a];
                int64_t i = ravel(&g, c);
                int64_t dlt = delta[i];
                if (dlt > -R && dlt < R) {
                    codes[i] = (uint16_t)(dlt + R);
                } else {
                    codes[i] = 0;
                    if (cnt < out_cap) {
                        out_idx[cnt] = (uint32_t)i;
                        out_val[cnt] = (int32_t)dlt;
                    }
                    ++cnt;
                }
            }
        }
        *n_out = cnt;
        if (cnt > out_cap) st = DQREF_ECAPACITY;
    }
    free(q);
    free(delta);
    return st;
}

/* ------------------------------------------------------------ decompress */

/* lexicographic (block id, local row-major position) order of two indices */
static int block_major_less(const geom *g, int64_t i, int64_t j) {
    int64_t ci[3], cj[3];
    unravel(g, i, ci);
    unravel(g, j, cj);
    int64_t bi = 0, bj = 0;
    for (int a = 0; a < g->d; ++a) {
        bi = bi * g->nb[a] + ci[a] / g->B;
        bj = bj * g->nb[a] + cj[a] / g->B;
    }
    if (bi != bj) return bi < bj;
    for (int a = 0; a < g->d; ++a) {
        int64_t li = ci[a] % g->B, lj = cj[a] % g->B;
        if (li != lj) return li < lj;
    }
    return 0;
}

int dqref_decompress(const dqref_params *p, double eb_abs, const uint16_t *codes,
                     const uint32_t *out_idx, const int32_t *out_val, uint64_t n_out,
                     const int32_t *pads, float *x_hat, int nthreads) {
    int st = dqref_validate(p);
    if (st != DQREF_OK) return st;
    if (!(eb_abs > 0.0) || !isfinite(eb_abs)) return DQREF_EINVAL;
    geom g;
    make_geom(p, &g);
    const int64_t R = p->radius;
    int32_t *delta = (int32_t *)malloc((size_t)g.N * sizeof(int32_t));
    int32_t *q = (int32_t *)malloc((size_t)g.N * sizeof(int32_t));
    unsigned char *have = (unsigned char *)calloc((size_t)g.N, 1);
    if (!delta || !q || !have) {
        free(delta);
        free(q);
        free(have);
        return DQREF_EINVAL;
    }
    for (int64_t i = 0; i < g.N; ++i) {
        if (codes[i] != 0) {
            delta[i] = (int32_t)((int64_t)codes[i] - R);
            have[i] = 1;
        }
    }
    for (uint64_t k = 0; k < n_out && st == DQREF_OK; ++k) {
        int64_t i = out_idx[k];
        if (i >= g.N || codes[i] != 0 || have[i]) st = DQREF_ECORRUPT;
        else if (k > 0 && !block_major_less(&g, out_idx[k - 1], i)) st = DQREF_ECORRUPT;
        else {
            delta[i] = out_val[k];
            have[i] = 1;
        }
    }
    for (int64_t i = 0; i < g.N && st == DQREF_OK; ++i)
        if (!have[i]) st = DQREF_ECORRUPT;
    if (st == DQREF_OK) st = dqref_reconstruct(p, delta, pads, q, nthreads);
    if (st == DQREF_OK) {
        const double two_eb = 2.0 * eb_abs;
        for (int64_t i = 0; i < g.N; ++i) {
            volatile double v = (double)q[i] * two_eb;
            x_hat[i] = (float)v;
        }
    }
    free(delta);
    free(q);
    free(have);
    return st;
}
