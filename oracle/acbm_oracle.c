/*
 * acbm_oracle.c -- plain CPU oracle for adaptive cost block matching.
 *
 * TEST INFRASTRUCTURE ONLY (see acbm_oracle.h).  Written for a reader holding
 * the paper: every function restates one definition or one step of the method
 * in the paper's order, with plain loops and exact integer arithmetic.  No
 * blocking, no pruning, no reordering.
 */
#include "acbm_oracle.h"

#include <stddef.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

void oracle_result_layout(uint32_t out[9])
{
    out[0] = (uint32_t)offsetof(oracle_result, mv_x);
    out[1] = (uint32_t)offsetof(oracle_result, mv_y);
    out[2] = (uint32_t)offsetof(oracle_result, sad);
    out[3] = (uint32_t)offsetof(oracle_result, j);
    out[4] = (uint32_t)offsetof(oracle_result, rate_bits);
    out[5] = (uint32_t)offsetof(oracle_result, cands);
    out[6] = (uint32_t)offsetof(oracle_result, mode);
    out[7] = (uint32_t)offsetof(oracle_result, intra_x);
    out[8] = (uint32_t)sizeof(oracle_result);
}

/* ------------------------------------------------------------------------ */
/* Geometry (Section 1): the current frame is cut into N x M blocks; the     */
/* candidate blocks live in the previous frame.  Frames must be whole        */
/* multiples of the block size; p is bounded so that a window index fits in  */
/* 16 bits.                                                                  */
/* ------------------------------------------------------------------------ */
int oracle_check_geom(const oracle_geom* g)
{
    if (!g) return ORACLE_EINVAL;
    if (g->width == 0 || g->height == 0 || g->block_w == 0 || g->block_h == 0)
        return ORACLE_EINVAL;
    if (g->pitch < g->width) return ORACLE_EINVAL;
    if (g->width % g->block_w != 0 || g->height % g->block_h != 0) return ORACLE_ESHAPE;
    if (g->p > 127) return ORACLE_ESHAPE;
    return ORACLE_OK;
}

static int blocks_x(const oracle_geom* g) { return (int)(g->width / g->block_w); }
static int blocks_y(const oracle_geom* g) { return (int)(g->height / g->block_h); }

/* ------------------------------------------------------------------------ */
/* Rate term R (Section 2.1; vectors are sent differentially, Section 2.2).  */
/* The paper names no code table.  The bit count used here is the length of  */
/* the signed Exp-Golomb codeword of one vector component: the signed value  */
/* k is mapped to code = 2k-1 (k > 0) or -2k (k <= 0), and the unsigned      */
/* Exp-Golomb codeword of `code` is (n-1) zero bits followed by the n-bit    */
/* binary form of code+1.                                                    */
/* ------------------------------------------------------------------------ */
int oracle_se_bits(int64_t k)
{
    uint64_t code = (k > 0) ? (uint64_t)(2 * k - 1) : (uint64_t)(-2 * k);
    uint64_t x = code + 1;
    int n = 0;
    while (x != 0) {
        n++;
        x >>= 1;
    }
    return 2 * n - 1;
}

/* ------------------------------------------------------------------------ */
/* Candidate validity.  The search area lies inside the previous frame        */
/* (Section 1), so a displaced block must be wholly inside the reference      */
/* frame and each component is bounded by p.                                 */
/* ------------------------------------------------------------------------ */
int oracle_is_valid(const oracle_geom* g, int r, int c, int u, int v)
{
    long p = (long)g->p;
    long x0 = (long)c * g->block_w, y0 = (long)r * g->block_h;
    if (u < -p || u > p || v < -p || v > p) return 0;
    if (x0 + u < 0 || x0 + u + (long)g->block_w > (long)g->width) return 0;
    if (y0 + v < 0 || y0 + v + (long)g->block_h > (long)g->height) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* SAD distortion (Section 2.1, SAD equation): sum over the block's pixels   */
/* of |p_t(i,j) - p_{t-1}(i+mv_x, j+mv_y)|, i horizontal (< N), j vertical   */
/* (< M).                                                                    */
/* ------------------------------------------------------------------------ */
uint32_t oracle_sad(const oracle_geom* g, const uint8_t* cur, const uint8_t* ref,
                    int r, int c, int u, int v)
{
    long x0 = (long)c * g->block_w, y0 = (long)r * g->block_h;
    uint32_t s = 0;
    for (long j = 0; j < (long)g->block_h; j++) {
        for (long i = 0; i < (long)g->block_w; i++) {
            int a = cur[(y0 + j) * g->pitch + (x0 + i)];
            int b = ref[(y0 + j + v) * g->pitch + (x0 + i + u)];
            s += (uint32_t)abs(a - b);
        }
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Half-pel precision (Section 2.2: the PBM refinement normally works on the */
/* half-pixel grid; Table 1's 969 full-search positions at p = 15 are the    */
/* 961 integer ones plus 8 half-pel ones).  The paper's simulations use an   */
/* H.263 coder (Section 4), so the half-pel reference is H.263's bilinear    */
/* interpolation: at half-pel coordinates (X, Y) = (2x + fx, 2y + fy)        */
/*   fx = fy = 0: A                                                          */
/*   fx = 1, fy = 0: (A + B + 1) / 2        fx = 0, fy = 1: (A + C + 1) / 2  */
/*   fx = fy = 1: (A + B + C + D + 2) / 4                                    */
/* with A = ref(x, y), B = ref(x+1, y), C = ref(x, y+1), D = ref(x+1, y+1)   */
/* and integer division (all terms are >= 0).                                */
/* ------------------------------------------------------------------------ */
static long half_floor(long X) { return X >= 0 ? X / 2 : -((-X + 1) / 2); }

int oracle_ref_half(const oracle_geom* g, const uint8_t* ref, long X, long Y)
{
    long x = half_floor(X), y = half_floor(Y);
    int fx = (int)(X - 2 * x), fy = (int)(Y - 2 * y);
    int A = ref[y * g->pitch + x];
    if (!fx && !fy) return A;
    if (fx && !fy) return (A + ref[y * g->pitch + x + 1] + 1) / 2;
    if (!fx && fy) return (A + ref[(y + 1) * g->pitch + x] + 1) / 2;
    return (A + ref[y * g->pitch + x + 1] + ref[(y + 1) * g->pitch + x] +
            ref[(y + 1) * g->pitch + x + 1] + 2) / 4;
}

/* A half-pel candidate (U, V) (units of half a pixel) is valid when each    */
/* component is within the window (|U|, |V| <= 2p) and every reference pixel */
/* the interpolation reads lies inside the frame.  Pixel (i, j) of the block */
/* reads columns floor((2(x0+i) + U)/2) and, when U is odd, the next one;    */
/* the extremes are i = 0 and i = N-1 (rows likewise).                       */
int oracle_is_valid_half(const oracle_geom* g, int r, int c, int U, int V)
{
    long p2 = 2 * (long)g->p;
    long x0 = (long)c * g->block_w, y0 = (long)r * g->block_h;
    if (U < -p2 || U > p2 || V < -p2 || V > p2) return 0;
    long xlo = half_floor(2 * x0 + U);
    long xhi = half_floor(2 * (x0 + (long)g->block_w - 1) + U) + (U & 1 ? 1 : 0);
    long ylo = half_floor(2 * y0 + V);
    long yhi = half_floor(2 * (y0 + (long)g->block_h - 1) + V) + (V & 1 ? 1 : 0);
    return xlo >= 0 && xhi <= (long)g->width - 1 && ylo >= 0 && yhi <= (long)g->height - 1;
}

/* SAD of a half-pel candidate: the SAD equation of Section 2.1 with the     */
/* candidate pixel taken from the half-pel reference.                        */
uint32_t oracle_sad_half(const oracle_geom* g, const uint8_t* cur, const uint8_t* ref,
                         int r, int c, int U, int V)
{
    long x0 = (long)c * g->block_w, y0 = (long)r * g->block_h;
    uint32_t s = 0;
    for (long j = 0; j < (long)g->block_h; j++) {
        for (long i = 0; i < (long)g->block_w; i++) {
            int a = cur[(y0 + j) * g->pitch + (x0 + i)];
            int b = oracle_ref_half(g, ref, 2 * (x0 + i) + U, 2 * (y0 + j) + V);
            s += (uint32_t)abs(a - b);
        }
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Intra_SAD (Section 3.1): sum of |p_t(i,j) - mu| with mu the block mean.   */
/* mu = S/(NM) is rational; multiplying every term by NM keeps it exact:     */
/* IntraX = NM * Intra_SAD = sum |NM * p_t(i,j) - S|.                        */
/* ------------------------------------------------------------------------ */
uint64_t oracle_intra_x(const oracle_geom* g, const uint8_t* cur, int r, int c)
{
    long x0 = (long)c * g->block_w, y0 = (long)r * g->block_h;
    int64_t nm = (int64_t)g->block_w * g->block_h;
    int64_t s = 0;
    for (long j = 0; j < (long)g->block_h; j++)
        for (long i = 0; i < (long)g->block_w; i++)
            s += cur[(y0 + j) * g->pitch + (x0 + i)];
    uint64_t acc = 0;
    for (long j = 0; j < (long)g->block_h; j++) {
        for (long i = 0; i < (long)g->block_w; i++) {
            int64_t d = nm * (int64_t)cur[(y0 + j) * g->pitch + (x0 + i)] - s;
            acc += (uint64_t)(d < 0 ? -d : d);
        }
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Median predictor.  Vectors are coded against a predictor built from      */
/* already coded neighbours (Section 2.2 says only causal neighbours exist). */
/* Neighbours: A left, B top, C top-right.  A missing left neighbour counts  */
/* as (0,0); on the first block row B and C take A's value; a missing        */
/* top-right neighbour (last column) counts as (0,0).  The predictor is the  */
/* component-wise median of A, B, C.                                         */
/* ------------------------------------------------------------------------ */
static int median3(int a, int b, int c)
{
    int v[3] = {a, b, c};
    /* three-element insertion sort, then the middle one */
    for (int i = 1; i < 3; i++) {
        int x = v[i], k = i - 1;
        while (k >= 0 && v[k] > x) {
            v[k + 1] = v[k];
            k--;
        }
        v[k + 1] = x;
    }
    return v[1];
}

void oracle_median_pred(const int32_t* fx, const int32_t* fy, int bx, int r, int c,
                        int* px, int* py)
{
    int ax = 0, ay = 0, bxv, byv, cx, cy;
    if (c > 0) {
        ax = fx[r * bx + (c - 1)];
        ay = fy[r * bx + (c - 1)];
    }
    if (r == 0) {
        bxv = ax; byv = ay;
        cx = ax;  cy = ay;
    } else {
        bxv = fx[(r - 1) * bx + c];
        byv = fy[(r - 1) * bx + c];
        if (c == bx - 1) {
            cx = 0; cy = 0;
        } else {
            cx = fx[(r - 1) * bx + (c + 1)];
            cy = fy[(r - 1) * bx + (c + 1)];
        }
    }
    *px = median3(ax, bxv, cx);
    *py = median3(ay, byv, cy);
}

/* ------------------------------------------------------------------------ */
/* Lagrangian cost (Section 2.1): J = SAD + lambda * R.  Ties in J are       */
/* broken by the smaller |u|+|v|, then by the earlier position in raster     */
/* order of the (2p+1)x(2p+1) window (mv_y outer, top-left first), so every  */
/* minimum is unique.                                                        */
/* ------------------------------------------------------------------------ */
typedef struct cand_eval {
    int u, v;
    uint32_t sad;
    uint32_t rate;
    uint64_t j;
    uint32_t l1;
    uint32_t raster;
} cand_eval;

/* Vectors are in units of 1/s pixel: s = 1 (integer) or s = 2 (half-pel).  */
/* The rate, the |u|+|v| tie-break and the raster position are all taken in  */
/* those units (the half-pel window is (4p+1) x (4p+1)).                     */
static int units(const oracle_params* prm) { return prm->subpel ? 2 : 1; }

static int valid_in_units(const oracle_geom* g, const oracle_params* prm, int r, int c,
                          int u, int v)
{
    return prm->subpel ? oracle_is_valid_half(g, r, c, u, v) : oracle_is_valid(g, r, c, u, v);
}

static cand_eval evaluate(const oracle_geom* g, const oracle_params* prm,
                          const uint8_t* cur, const uint8_t* ref, int r, int c,
                          int u, int v, int px, int py)
{
    cand_eval e;
    int sp = units(prm) * (int)g->p;
    e.u = u;
    e.v = v;
    e.sad = prm->subpel ? oracle_sad_half(g, cur, ref, r, c, u, v)
                        : oracle_sad(g, cur, ref, r, c, u, v);
    e.rate = (uint32_t)(oracle_se_bits((int64_t)u - px) + oracle_se_bits((int64_t)v - py));
    e.j = (uint64_t)e.sad + (uint64_t)prm->lambda * e.rate;
    e.l1 = (uint32_t)(abs(u) + abs(v));
    e.raster = (uint32_t)((v + sp) * (2 * sp + 1) + (u + sp));
    return e;
}

static int cheaper(const cand_eval* a, const cand_eval* b)
{
    if (a->j != b->j) return a->j < b->j;
    if (a->l1 != b->l1) return a->l1 < b->l1;
    return a->raster < b->raster;
}

static void store(oracle_result* o, const cand_eval* e, uint32_t cands, uint32_t mode,
                  uint64_t intra_x)
{
    o->mv_x = e->u;
    o->mv_y = e->v;
    o->sad = e->sad;
    o->j = e->j;
    o->rate_bits = e->rate;
    o->cands = cands;
    o->mode = mode;
    o->intra_x = intra_x;
}

/* Full search over the window of one block (Section 2.3): every valid       */
/* integer position is evaluated and the cheapest kept.  With half-pel       */
/* precision the 8 half-pel positions around that winner are evaluated next  */
/* (Table 1 counts them: 969 = 31^2 + 8 at p = 15) and the cheapest of all   */
/* is the result.  Returns the number of positions evaluated.                */
static uint32_t full_search(const oracle_geom* g, const oracle_params* prm,
                            const uint8_t* cur, const uint8_t* ref, int r, int c,
                            int px, int py, cand_eval* best)
{
    int p = (int)g->p, s = units(prm);
    uint32_t count = 0;
    for (int v = -p; v <= p; v++) {
        for (int u = -p; u <= p; u++) {
            if (!oracle_is_valid(g, r, c, u, v)) continue;
            cand_eval e = evaluate(g, prm, cur, ref, r, c, s * u, s * v, px, py);
            if (count == 0 || cheaper(&e, best)) *best = e;
            count++;
        }
    }
    if (prm->subpel) {
        int cu = best->u, cv = best->v; /* the integer winner, on the even grid */
        for (int dv = -1; dv <= 1; dv++) {
            for (int du = -1; du <= 1; du++) {
                if (du == 0 && dv == 0) continue;
                if (!oracle_is_valid_half(g, r, c, cu + du, cv + dv)) continue;
                cand_eval e = evaluate(g, prm, cur, ref, r, c, cu + du, cv + dv, px, py);
                if (cheaper(&e, best)) *best = e;
                count++;
            }
        }
    }
    return count;
}

/* ------------------------------------------------------------------------ */
/* SAD table and Intra table.                                                */
/* ------------------------------------------------------------------------ */
int oracle_sad_table(const oracle_geom* g, const uint8_t* cur, const uint8_t* ref,
                     uint32_t* table)
{
    int rc = oracle_check_geom(g);
    if (rc) return rc;
    if (!cur || !ref || !table) return ORACLE_EINVAL;
    int p = (int)g->p, w = 2 * p + 1;
    int bx = blocks_x(g), by = blocks_y(g);
    for (int r = 0; r < by; r++)
        for (int c = 0; c < bx; c++)
            for (int v = -p; v <= p; v++)
                for (int u = -p; u <= p; u++) {
                    size_t at = (((size_t)r * bx + c) * w + (v + p)) * w + (u + p);
                    table[at] = oracle_is_valid(g, r, c, u, v)
                                    ? oracle_sad(g, cur, ref, r, c, u, v)
                                    : 0xFFFFFFFFu;
                }
    return ORACLE_OK;
}

int oracle_intra_table(const oracle_geom* g, const uint8_t* cur, uint64_t* intra_x)
{
    int rc = oracle_check_geom(g);
    if (rc) return rc;
    if (!cur || !intra_x) return ORACLE_EINVAL;
    int bx = blocks_x(g), by = blocks_y(g);
    for (int r = 0; r < by; r++)
        for (int c = 0; c < bx; c++)
            intra_x[r * bx + c] = oracle_intra_x(g, cur, r, c);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* FSBM for one frame pair (Section 2.3), blocks in raster order so that    */
/* each block's predictor uses the final vectors of its causal neighbours.  */
/* ------------------------------------------------------------------------ */
static int check_params(const oracle_params* prm)
{
    if (!prm) return ORACLE_EINVAL;
    if (prm->gamma_den == 0) return ORACLE_EINVAL;
    if (prm->subpel > 1) return ORACLE_EINVAL;
    return ORACLE_OK;
}

int oracle_fsbm_frame(const oracle_geom* g, const oracle_params* prm,
                      const uint8_t* cur, const uint8_t* ref, oracle_result* out)
{
    int rc = oracle_check_geom(g);
    if (rc) return rc;
    if ((rc = check_params(prm))) return rc;
    if (!cur || !ref || !out) return ORACLE_EINVAL;
    int bx = blocks_x(g), by = blocks_y(g);
    int32_t* fx = calloc((size_t)bx * by, sizeof(int32_t));
    int32_t* fy = calloc((size_t)bx * by, sizeof(int32_t));
    if (!fx || !fy) {
        free(fx);
        free(fy);
        return ORACLE_EINVAL;
    }
    for (int r = 0; r < by; r++) {
        for (int c = 0; c < bx; c++) {
            int px, py;
            oracle_median_pred(fx, fy, bx, r, c, &px, &py);
            cand_eval best;
            uint32_t n = full_search(g, prm, cur, ref, r, c, px, py, &best);
            store(&out[r * bx + c], &best, n, 0, oracle_intra_x(g, cur, r, c));
            fx[r * bx + c] = best.u;
            fy[r * bx + c] = best.v;
        }
    }
    free(fx);
    free(fy);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* PBM for one block (Section 2.2), three steps:                             */
/*  1. the predictor set: (0,0); the final vectors of the causal spatial     */
/*     neighbours left, top-left, top, top-right in this frame; the previous */
/*     field at the co-located block and its eight neighbours.  Neighbours   */
/*     outside the block grid are absent; predictors that are not valid      */
/*     candidates for this block are dropped; repeats count once.            */
/*  2. the cheapest predictor;                                               */
/*  3. one refinement step: the valid 8-neighbours of that predictor on the */
/*     finest grid in use (integer, or half-pel with subpel: "normally" the  */
/*     half-pixel grid, Section 2.2) not already evaluated, then the         */
/*     cheapest of everything.  Vectors of the fields are in the same units. */
/* ------------------------------------------------------------------------ */
#define MAX_SET 32

static int in_set(const cand_eval* set, int n, int u, int v)
{
    for (int k = 0; k < n; k++)
        if (set[k].u == u && set[k].v == v) return 1;
    return 0;
}

static void pbm_block(const oracle_geom* g, const oracle_params* prm,
                      const uint8_t* cur, const uint8_t* ref, const int16_t* prev_field,
                      const int32_t* fx, const int32_t* fy, int r, int c, int px, int py,
                      cand_eval* best, uint32_t* cands)
{
    int bx = blocks_x(g), by = blocks_y(g);
    int pu[MAX_SET], pv[MAX_SET], np = 0;

    /* step 1: gather the raw predictors */
    pu[np] = 0; pv[np] = 0; np++;
    const int sdr[4] = {0, -1, -1, -1}, sdc[4] = {-1, -1, 0, 1}; /* L, TL, T, TR */
    for (int k = 0; k < 4; k++) {
        int rr = r + sdr[k], cc = c + sdc[k];
        if (rr < 0 || cc < 0 || cc >= bx) continue;
        pu[np] = fx[rr * bx + cc];
        pv[np] = fy[rr * bx + cc];
        np++;
    }
    for (int dr = -1; dr <= 1; dr++) {
        for (int dc = -1; dc <= 1; dc++) {
            int rr = r + dr, cc = c + dc;
            if (rr < 0 || rr >= by || cc < 0 || cc >= bx) continue;
            pu[np] = prev_field ? prev_field[2 * (rr * bx + cc) + 0] : 0;
            pv[np] = prev_field ? prev_field[2 * (rr * bx + cc) + 1] : 0;
            np++;
        }
    }

    /* step 1 (cont.): keep valid, distinct predictors and evaluate them */
    cand_eval set[MAX_SET];
    int n = 0;
    for (int k = 0; k < np; k++) {
        if (!valid_in_units(g, prm, r, c, pu[k], pv[k])) continue;
        if (in_set(set, n, pu[k], pv[k])) continue;
        set[n++] = evaluate(g, prm, cur, ref, r, c, pu[k], pv[k], px, py);
    }

    /* step 2: the cheapest predictor */
    cand_eval b0 = set[0];
    for (int k = 1; k < n; k++)
        if (cheaper(&set[k], &b0)) b0 = set[k];

    /* step 3: refinement around it, one step of the finest grid */
    for (int dv = -1; dv <= 1; dv++) {
        for (int du = -1; du <= 1; du++) {
            if (du == 0 && dv == 0) continue;
            int u = b0.u + du, v = b0.v + dv;
            if (!valid_in_units(g, prm, r, c, u, v)) continue;
            if (in_set(set, n, u, v)) continue;
            set[n++] = evaluate(g, prm, cur, ref, r, c, u, v, px, py);
        }
    }
    cand_eval b = set[0];
    for (int k = 1; k < n; k++)
        if (cheaper(&set[k], &b)) b = set[k];
    *best = b;
    *cands = (uint32_t)n;
}

/* ACBM decision (Section 3.2) for a block with Intra_SAD = intra/(N*M) and
 * PBM result SAD sad_p.  First test: Intra_SAD + SAD_PBM < alpha + beta*Qp^2;
 * second test: SAD_PBM < gamma * Intra_SAD.  Both are multiplied through by
 * N*M (and gamma_den) so that Intra_SAD stays exact.  Returns 1 or 2 for the
 * test that kept PBM, 3 for a critical block. */
static int acbm_decide(const oracle_geom* g, const oracle_params* prm, uint64_t intra,
                       uint32_t sad_p)
{
    u128 nm = (u128)g->block_w * g->block_h;
    u128 t1 = (u128)prm->alpha + (u128)prm->beta * prm->qp * prm->qp;
    int c1 = (u128)intra + nm * sad_p < nm * t1;
    int c2 = (u128)prm->gamma_den * nm * sad_p < (u128)prm->gamma_num * intra;
    if (c1) return 1;
    if (c2) return 2;
    return 3;
}

/* Shared frame loop of the PBM and ACBM runs. */
static int predictive_frame(const oracle_geom* g, const oracle_params* prm,
                            const uint8_t* cur, const uint8_t* ref,
                            const int16_t* prev_field, oracle_result* out, int acbm)
{
    int rc = oracle_check_geom(g);
    if (rc) return rc;
    if ((rc = check_params(prm))) return rc;
    if (!cur || !ref || !out) return ORACLE_EINVAL;
    int bx = blocks_x(g), by = blocks_y(g);
    int32_t* fx = calloc((size_t)bx * by, sizeof(int32_t));
    int32_t* fy = calloc((size_t)bx * by, sizeof(int32_t));
    if (!fx || !fy) {
        free(fx);
        free(fy);
        return ORACLE_EINVAL;
    }
    for (int r = 0; r < by; r++) {
        for (int c = 0; c < bx; c++) {
            int px, py;
            oracle_median_pred(fx, fy, bx, r, c, &px, &py);
            /* Section 3.2: Intra_SAD first, then PBM */
            uint64_t intra = oracle_intra_x(g, cur, r, c);
            cand_eval pbm;
            uint32_t cands;
            pbm_block(g, prm, cur, ref, prev_field, fx, fy, r, c, px, py, &pbm, &cands);
            oracle_result* o = &out[r * bx + c];
            if (!acbm) {
                store(o, &pbm, cands, 4, intra);
            } else {
                int mode = acbm_decide(g, prm, intra, pbm.sad);
                if (mode != 3) {
                    store(o, &pbm, cands, (uint32_t)mode, intra);
                } else {
                    /* critical block: full search with the same predictor */
                    cand_eval fs;
                    uint32_t n = full_search(g, prm, cur, ref, r, c, px, py, &fs);
                    store(o, &fs, cands + n, 3, intra);
                }
            }
            fx[r * bx + c] = o->mv_x;
            fy[r * bx + c] = o->mv_y;
        }
    }
    free(fx);
    free(fy);
    return ORACLE_OK;
}

int oracle_block(const oracle_geom* g, const oracle_params* prm, int algo,
                 const uint8_t* cur, const uint8_t* ref, const int16_t* prev_field,
                 const int32_t* field_x, const int32_t* field_y, int r, int c,
                 oracle_result* out)
{
    int rc = oracle_check_geom(g);
    if (rc) return rc;
    if ((rc = check_params(prm))) return rc;
    if (!cur || !ref || !field_x || !field_y || !out) return ORACLE_EINVAL;
    if (r < 0 || c < 0 || r >= blocks_y(g) || c >= blocks_x(g)) return ORACLE_EINVAL;
    int px, py;
    oracle_median_pred(field_x, field_y, blocks_x(g), r, c, &px, &py);
    uint64_t intra = oracle_intra_x(g, cur, r, c);
    if (algo == ORACLE_FSBM) {
        cand_eval best;
        uint32_t count = full_search(g, prm, cur, ref, r, c, px, py, &best);
        store(out, &best, count, 0, intra);
        return ORACLE_OK;
    }
    cand_eval pbm;
    uint32_t npbm;
    pbm_block(g, prm, cur, ref, prev_field, field_x, field_y, r, c, px, py, &pbm, &npbm);
    if (algo == ORACLE_PBM) {
        store(out, &pbm, npbm, 4, intra);
        return ORACLE_OK;
    }
    int mode = acbm_decide(g, prm, intra, pbm.sad);
    if (mode != 3) {
        store(out, &pbm, npbm, (uint32_t)mode, intra);
    } else {
        cand_eval whole;
        uint32_t nwin = full_search(g, prm, cur, ref, r, c, px, py, &whole);
        store(out, &whole, npbm + nwin, 3, intra);
    }
    return ORACLE_OK;
}

int oracle_pbm_frame(const oracle_geom* g, const oracle_params* prm,
                     const uint8_t* cur, const uint8_t* ref,
                     const int16_t* prev_field, oracle_result* out)
{
    return predictive_frame(g, prm, cur, ref, prev_field, out, 0);
}

int oracle_acbm_frame(const oracle_geom* g, const oracle_params* prm,
                      const uint8_t* cur, const uint8_t* ref,
                      const int16_t* prev_field, oracle_result* out)
{
    return predictive_frame(g, prm, cur, ref, prev_field, out, 1);
}

/* ------------------------------------------------------------------------ */
/* Sequences: pair t uses frame t-1 as reference; the predictive searches   */
/* take the previous pair's field as their temporal neighbourhood (all zero */
/* for the first pair).                                                     */
/* ------------------------------------------------------------------------ */
int oracle_sequence(const oracle_geom* g, const oracle_params* prm, int algo,
                    const uint8_t* const* frames, uint32_t nframes, oracle_result* out)
{
    int rc = oracle_check_geom(g);
    if (rc) return rc;
    if (!frames || !out || nframes < 2) return ORACLE_EINVAL;
    if (algo != ORACLE_FSBM && algo != ORACLE_PBM && algo != ORACLE_ACBM) return ORACLE_EINVAL;
    size_t nb = (size_t)blocks_x(g) * blocks_y(g);
    int16_t* prev = NULL;
    for (uint32_t t = 1; t < nframes; t++) {
        oracle_result* o = out + (t - 1) * nb;
        if (algo == ORACLE_FSBM)
            rc = oracle_fsbm_frame(g, prm, frames[t], frames[t - 1], o);
        else if (algo == ORACLE_PBM)
            rc = oracle_pbm_frame(g, prm, frames[t], frames[t - 1], prev, o);
        else
            rc = oracle_acbm_frame(g, prm, frames[t], frames[t - 1], prev, o);
        if (rc) break;
        if (!prev) prev = malloc(nb * 2 * sizeof(int16_t));
        if (!prev) return ORACLE_EINVAL;
        for (size_t b = 0; b < nb; b++) {
            prev[2 * b + 0] = (int16_t)o[b].mv_x;
            prev[2 * b + 1] = (int16_t)o[b].mv_y;
        }
    }
    free(prev);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* SAD_deviation (Section 3.1): sum over the evaluated positions of          */
/* |SAD(u,v) - SAD_min|, with SAD_min the smallest SAD among them.  Here the */
/* evaluated positions are the full valid window.                            */
/* ------------------------------------------------------------------------ */
int oracle_sad_deviation(const oracle_geom* g, const uint8_t* cur, const uint8_t* ref,
                         int r, int c, uint64_t* deviation, uint32_t* sad_min)
{
    int rc = oracle_check_geom(g);
    if (rc) return rc;
    if (!cur || !ref || !deviation || !sad_min) return ORACLE_EINVAL;
    int p = (int)g->p;
    uint32_t mn = 0xFFFFFFFFu;
    for (int v = -p; v <= p; v++)
        for (int u = -p; u <= p; u++)
            if (oracle_is_valid(g, r, c, u, v)) {
                uint32_t s = oracle_sad(g, cur, ref, r, c, u, v);
                if (s < mn) mn = s;
            }
    uint64_t dev = 0;
    for (int v = -p; v <= p; v++)
        for (int u = -p; u <= p; u++)
            if (oracle_is_valid(g, r, c, u, v))
                dev += oracle_sad(g, cur, ref, r, c, u, v) - mn;
    *deviation = dev;
    *sad_min = mn;
    return ORACLE_OK;
}
