/*
 * acbm_oracle.h -- plain CPU oracle for adaptive cost block matching (ACBM).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a slow, obviously correct restatement of the method.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does.  It shares no code, header, table or constant with
 * the GPU library.
 *
 * Method: S. Lopez, G.M. Callico, J.F. Lopez, R. Sarmiento, "A High
 * Quality/Low Computational Cost Technique for Block Matching Motion
 * Estimation".  Section numbers below refer to that paper.
 *
 * Everything is integer and exact.  Conventions where the paper is silent are
 * the readings listed in the design notes (frame border, median predictor,
 * rate code, tie-break, PBM candidate set); each function names the one it
 * uses.
 */
#ifndef ACBM_ORACLE_H
#define ACBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Frame and block geometry (Section 1).  Frames are u8 luma, row-major with a
 * row pitch in bytes.  block_w is N (pairs with mv_x), block_h is M (pairs
 * with mv_y), p is the maximum displacement. */
typedef struct oracle_geom {
    uint32_t width, height, pitch;
    uint32_t block_w, block_h;
    uint32_t p;
} oracle_geom;

/* Lagrange multiplier and the ACBM thresholds (Sections 2.1 and 3.2).
 * gamma = gamma_num / gamma_den.  subpel = 1 selects half-pel precision
 * (Section 2.2's refinement on the half-pixel grid, and the 8 half-pel
 * positions of the full search counted in Table 1): every vector, predictor
 * and rate is then in half-pel units. */
typedef struct oracle_params {
    uint32_t lambda, qp;
    uint32_t alpha, beta;
    uint32_t gamma_num, gamma_den;
    uint32_t subpel;
} oracle_params;

/* One block's outcome.  Deliberately a different layout from the GPU
 * library's result record: tests compare field by field. */
typedef struct oracle_result {
    int32_t  mv_x, mv_y;
    uint32_t sad;        /* SAD of the chosen vector                      */
    uint64_t j;          /* J = SAD + lambda * R                          */
    uint32_t rate_bits;  /* R: bits of the differential vector            */
    uint32_t cands;      /* candidate positions evaluated for this block  */
    uint32_t mode;       /* 0 FSBM, 1 PBM accepted by the first test,
                            2 PBM accepted by the second test,
                            3 critical (full search), 4 plain PBM run     */
    uint64_t intra_x;    /* N*M*Intra_SAD, exact                          */
} oracle_result;

enum { ORACLE_FSBM = 0, ORACLE_PBM = 1, ORACLE_ACBM = 2 };

/* Status codes of the oracle (its own; only zero / non-zero matters). */
enum { ORACLE_OK = 0, ORACLE_EINVAL = -1, ORACLE_ESHAPE = -2 };

/* Byte offsets of the oracle_result fields followed by its size, so that a
 * caller can describe the record without guessing the compiler's padding:
 * mv_x, mv_y, sad, j, rate_bits, cands, mode, intra_x, sizeof. */
void     oracle_result_layout(uint32_t out[9]);

int      oracle_check_geom(const oracle_geom* g);
int      oracle_se_bits(int64_t k);
int      oracle_is_valid(const oracle_geom* g, int r, int c, int u, int v);
uint32_t oracle_sad(const oracle_geom* g, const uint8_t* cur, const uint8_t* ref,
                    int r, int c, int u, int v);
uint64_t oracle_intra_x(const oracle_geom* g, const uint8_t* cur, int r, int c);
/* Half-pel sample of the reference at half-pel coordinates (X, Y) = (2x + fx,
 * 2y + fy) (bilinear, rounding as H.263), and the SAD and validity of a
 * half-pel candidate (U, V) of block (r, c). */
int      oracle_ref_half(const oracle_geom* g, const uint8_t* ref, long X, long Y);
int      oracle_is_valid_half(const oracle_geom* g, int r, int c, int U, int V);
uint32_t oracle_sad_half(const oracle_geom* g, const uint8_t* cur, const uint8_t* ref,
                         int r, int c, int U, int V);
void     oracle_median_pred(const int32_t* field_x, const int32_t* field_y,
                            int bx, int r, int c, int* px, int* py);

/* Full table of SADs, layout [by][bx][2p+1][2p+1] (mv_y outer, mv_x inner),
 * 0xFFFFFFFF where the candidate is not valid. */
int oracle_sad_table(const oracle_geom* g, const uint8_t* cur, const uint8_t* ref,
                     uint32_t* table);

/* IntraX for every block, [by][bx]. */
int oracle_intra_table(const oracle_geom* g, const uint8_t* cur, uint64_t* intra_x);

/* One frame pair.  prev_field holds (x, y) int16 pairs per block of the
 * previous pair's result field; NULL means all zero. */
int oracle_fsbm_frame(const oracle_geom* g, const oracle_params* prm,
                      const uint8_t* cur, const uint8_t* ref, oracle_result* out);
int oracle_pbm_frame(const oracle_geom* g, const oracle_params* prm,
                     const uint8_t* cur, const uint8_t* ref,
                     const int16_t* prev_field, oracle_result* out);
int oracle_acbm_frame(const oracle_geom* g, const oracle_params* prm,
                      const uint8_t* cur, const uint8_t* ref,
                      const int16_t* prev_field, oracle_result* out);

/* A sequence of nframes frames gives nframes-1 pairs (frame t-1 is the
 * reference of frame t).  out holds (nframes-1) fields of by*bx results. */
int oracle_sequence(const oracle_geom* g, const oracle_params* prm, int algo,
                    const uint8_t* const* frames, uint32_t nframes,
                    oracle_result* out);

/* One block of a raster run, given the final vectors of the blocks before it
 * (field_x/field_y, [by][bx], only entries before (r, c) are read) and the
 * previous field: the block's FSBM (algo 0), PBM (1) or ACBM (2) result.
 * Used to check single blocks of frames too large for a whole raster run. */
int oracle_block(const oracle_geom* g, const oracle_params* prm, int algo,
                 const uint8_t* cur, const uint8_t* ref, const int16_t* prev_field,
                 const int32_t* field_x, const int32_t* field_y, int r, int c,
                 oracle_result* out);

/* Sum of |SAD(u,v) - SAD_min| over the valid window of one block
 * (Section 3.1, SAD_deviation) and the SAD minimum itself. */
int oracle_sad_deviation(const oracle_geom* g, const uint8_t* cur, const uint8_t* ref,
                         int r, int c, uint64_t* deviation, uint32_t* sad_min);

#ifdef __cplusplus
}
#endif
#endif
