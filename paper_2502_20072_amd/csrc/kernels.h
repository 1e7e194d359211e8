// Device-pointer view of a handle's workspace and the kernel launchers.
#pragma once

#include "common.h"

namespace sl0 {

struct Ctx {
    // problem (caller memory)
    const double *F;
    const double *y;
    int64_t n_total, S;
    int T, TP;
    int64_t Gnt;  // 64-wide tiles per row of the tiled correlation matrices
    int64_t rows_max;  // rows of the largest task (chooses the statistics kernels' form)
    // carved from the workspace
    int64_t *off_dev;
    int32_t *torder;                 // tasks by decreasing row count (the Gram's launch order)
    double *ybar, *cyy, *mu, *inv_s, *bhat, *G, *part;
    uint32_t *flags;
    int32_t *lp_cbase;               // precision form: first chunk of each task [T+1]
    int32_t *lp_exp;                 // precision form: chunk exponents [S][lp_nchunk]
    __bf16 *lp_slices;               // precision form: slices [NS][S][lp_nchunk * LP_XC]
    unsigned long long *err_bits;    // error report: max |G error| bit pattern
    unsigned long long *theta_bits;  // shared SSE bound (bit pattern of a non-negative double)
    unsigned int *work_counter;      // next search work item
    unsigned int *cand_counter;      // slow-path candidates seen (diagnostics)
    unsigned int *merge_count;       // merge: candidates appended
    uint64_t *stats;                 // [4]: candidates, work items, theta0 bits, final theta bits
    uint64_t *cum;                   // cumulative work items per j-block [S/JBLK + 2]
    uint64_t *btab;                  // binomials C(n, r), r <= SISSO_MAX_D, n <= S
    int32_t *pre_prefix;             // pre-pass: chosen prefixes [PRE_Q][SISSO_MAX_D]
    int32_t *pre_count;              // pre-pass: number of chosen prefixes
    unsigned int *pre_done;          // pre-pass: extension blocks finished (the last one pools)
    double *pre_sse;                 // pre-pass: extension scores [PRE_Q][S]
    double *pre_bound;               // pre-pass: per-prefix L-th best [PRE_Q]
    double *rec3;                    // D = 3: pair records of the filter task [ceil(S/4)][S][4][4] (null if absent)
    double *G1;                      // the filter task's matrix alone, one-task tiled layout (G itself when T = 1)
    double *rec4;                    // D = 4, one task: pair-group records [rows][S4_ROW] (null if absent)
    int64_t *r4off;                  //   record rows of the groups with i2 below each index [S + 1]
    uint64_t *mtq;                   // several tasks, D = 3: flagged sweep steps [mtq_chunks][MTQ_CHUNK][3]
    uint32_t *mtq_n;                 //   keys per chunk
    uint64_t *mtq_pre;               //   exclusive prefix of mtq_n over the chunks taken [+1]
    unsigned int *mtq_taken;         //   chunks taken from the pool (may run past mtq_chunks)
    int mtq_chunks;                  //   chunks in the pool (0: none)
    int32_t *tstar;                  // filter tasks [2]: the tasks of largest and second largest
                                     // |y_t - ybar_t|^2 (0 and -1 when T = 1)
    double *list_sse;                // per-wave lists [nwaves][KP]
    uint64_t *list_rank;
    double *cand_sse;                // merge: compacted candidates [nwaves * KP]
    uint64_t *cand_rank;
    double *merged_sse;              // [KP]
    uint64_t *merged_rank;
    double *resc_sse;                // rescored [KP]
    double *resc_coef;               // [KP][T][D_max+1]
    uint32_t *res_flags;             // final: copy of the status words [4], head of the result block
    int32_t *res_idx;                // final [k_max][D_max]
    double *res_sse;                 // [k_max]
    double *res_coef;                // [k_max][T][D_max+1]
    int nsplit, KP, nwaves, search_wgs, D_max, k_max;
    int lp_ns, lp_nchunk;            // precision form: slices per value (0 = FP64), chunks
    int fp32;                        // FP32 solve form: the sweep's per-tuple solves in FP32
    // host-side: start/stop events per phase when profiling is on (else null)
    hipEvent_t *ev;
};

inline void phase_begin(const Ctx &c, int ph, hipStream_t st) {
    if (c.ev) (void)hipEventRecord(c.ev[2 * ph], st);
}
inline void phase_end(const Ctx &c, int ph, hipStream_t st) {
    if (c.ev) (void)hipEventRecord(c.ev[2 * ph + 1], st);
}

// search parameters of one call
struct SearchCall {
    int D, k;
    int ranged;
    uint64_t r0, r1;
};

uint64_t s3_tiles_host(int64_t S);  // tiles of the D = 3 record-table sweep
int s3_rows_per_tile();             // rows j per tile of that sweep (its steps per tile, at most)
uint64_t s4_tiles_host(int64_t S);  // tiles of the D = 4 record-table sweep
int launch_stats(const Ctx &c, hipStream_t st);
int launch_gram(const Ctx &c, hipStream_t st);  // FP64 MFMA or precision form, then finish
int launch_gram_lp(const Ctx &c, int NS, hipStream_t st);
int launch_gram_check(const Ctx &c, int nsample, unsigned long long *out_bits, hipStream_t st);
int launch_untile(const Ctx &c, int t, double *dst, hipStream_t st);
int launch_search(const Ctx &c, const SearchCall &sc, hipStream_t st);
int launch_prefix_best(const Ctx &c, int M, const int32_t *pre, int64_t n, double *best, hipStream_t st);
int launch_prefix_target(const Ctx &c, const double *best, int64_t n, float *target, hipStream_t st);
int launch_prefix_features(const Ctx &c, int M, const int32_t *pre, int64_t n, float *out, hipStream_t st);
int launch_prefix_extend(const Ctx &c, int M, const int32_t *pre, int64_t n, int32_t *out, hipStream_t st);
int launch_prefix_features_range(const Ctx &c, int M, uint64_t r0, int64_t n, float *out, hipStream_t st);
int launch_list_search(const Ctx &c, int D, int k, const int32_t *pre, int64_t n, hipStream_t st);

// batched one-task D = 3 search: per-problem prologue, one search launch for
// all problems, per-problem epilogue (merge, re-score, final ordering)
constexpr int S3B_MAXP = 128;  // problems per batched search launch
constexpr int S3B_RUN = 16;    // consecutive tiles per queue item
struct BatchSearchArgs {
    int P;                          // problems, ordered by decreasing tile count
    int KPmax;                      // longest list among them
    const uint32_t *item_end;       // device [P]: inclusive prefix of the problems' item counts
    const Ctx *const *ctx;          // device [P]: each problem's Ctx, copied to its workspace
};
constexpr size_t S3B_TABLE_BYTES = S3B_MAXP * (sizeof(uint32_t) + sizeof(void *)) + 64;
bool s3_batchable(const Ctx &c, int D);
int launch_batch_prologue(const Ctx &c, const SearchCall &sc, hipStream_t st);
int launch_batch_search3(const BatchSearchArgs &b, int wgs, hipStream_t st);
int launch_batch_epilogue(const Ctx &c, const SearchCall &sc, hipStream_t st);

}  // namespace sl0
