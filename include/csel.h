/*
 * csel.h -- C ABI of the greedy conditional-selection library for MI355X (gfx950).
 *
 * The library builds sparse inverse-Cholesky factors of kernel covariance
 * matrices by greedy conditional selection (Huan, Guinness, Katzfuss, Owhadi,
 * Schaefer, "Sparse inverse Cholesky factorization of dense kernel matrices by
 * greedy conditional selection", arXiv:2307.11648).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers owned by the caller, unless the
 *    comment says "host".  Nothing is freed or retained across a call.
 *  - Work is enqueued asynchronously on `stream` (0 = the null stream);
 *    outputs are valid once the stream is synchronized.  Calls on one stream
 *    are ordered; the library keeps no per-call state between calls.
 *  - Points are given in ordering-position order: "later" means a larger
 *    index.  Coordinates are FP64, row-major [n][dim], 1 <= dim <= 3.
 *  - Return value: CSEL_OK or a negative csel_error.  Arguments that can be
 *    checked on the host are checked before anything is enqueued; the message
 *    of the last failure on the calling thread is in csel_last_error().
 *    Problems found inside a kernel (index out of range, numerical breakdown)
 *    are not errors of the call: they are reported per column in `status`.
 *  - Per-column status codes:
 *      0 ok
 *      1 stopped early: no candidate left with positive conditional variance;
 *        the factor is built on the candidates selected so far
 *      2 the selected covariance block was not numerically positive definite;
 *        the column's values are NaN
 *      3 bad input for this column (target or pool index outside [0, n),
 *        pool_len outside [0, pool_stride]); the column is left as for status 2
 *      4 (aggregated only) a pool index precedes a group member while factor
 *        values were requested
 *      5 (aggregated only) the aggregated pattern exceeds the factor block
 *        size; the selection outputs are valid, the columns are not written
 *  - No C++ exception crosses this boundary.
 */
#ifndef CSEL_H
#define CSEL_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CSEL_OK = 0,
    CSEL_EINVAL = -1,       /* an argument is invalid (see csel_last_error) */
    CSEL_EHIP = -2,         /* a HIP runtime call failed */
    CSEL_ENOMEM = -3,       /* device workspace could not be allocated */
    CSEL_EUNSUPPORTED = -4  /* valid request outside what the library supports */
} csel_error;

enum { CSEL_FP64 = 0, CSEL_MIXED = 1 };

/* Schedules of csel_aggregated_select_sched (see there). */
enum {
    CSEL_AGG_AUTO = 0,       /* the library's rule (csel_aggregated_select) */
    CSEL_AGG_ONE_GROUP = 1,  /* one workgroup per group */
    CSEL_AGG_REGISTER = 2,   /* the mixed register-resident kernel */
    CSEL_AGG_SPLIT_256 = 3,  /* a group's rows over workgroups of 256 threads */
    CSEL_AGG_SPLIT_512 = 4,  /* ... of 512 threads */
    CSEL_AGG_SPLIT_1024 = 5  /* ... of 1024 threads */
};

/* Matern covariance K(x, y) = variance * m_nu(|x - y| / length_scale) with
 * nu = two_nu / 2 in {1/2, 3/2, 5/2}, plus `nugget` on the diagonal (by
 * index).  The paper uses the Matern family throughout (Sec. 6) without
 * printing it; these are the textbook half-integer forms:
 *   nu=1/2: exp(-a), a = r/l;   nu=3/2: (1+a)exp(-a), a = sqrt(3) r/l;
 *   nu=5/2: (1+a+a^2/3)exp(-a), a = sqrt(5) r/l. */
typedef struct {
    int32_t two_nu;
    double length_scale; /* > 0 */
    double variance;     /* > 0 */
    double nugget;       /* >= 0 */
} csel_kernel;

/* Message for the last non-OK return on the calling thread ("" if none). */
const char *csel_last_error(void);

/* ABI version, currently 1. */
int32_t csel_version(void);

/* Largest pool size and number of selections per column the library handles
 * for csel_select_and_factor. */
int32_t csel_max_pool(void);
int32_t csel_max_select(void);

/*
 * csel_select_and_factor -- greedy single-target selection per column and its
 * KL-optimal factor column.
 *
 * For each target column i = targets[c] (Sec. 4): the candidates are
 * pool_idx[c*pool_stride + 0 .. pool_len[c]) (ids of later points, sorted by
 * distance, ascending).  k_c = min(k, pool_len[c]) points are selected one at
 * a time, each maximizing the decrease of the target's conditional variance,
 * cov(i, j | I)^2 / var(j | I) (eq. obj_gp), with the conditional variances
 * and covariances kept by rank-one downdates of a partial Cholesky factor
 * (eq. cond_select; App. C.1).  A candidate stays eligible while its
 * conditional variance exceeds 1e-12 times its prior variance.  Ties in score
 * go to the smaller pool slot.  The column on s = [i, selected...] is then
 * L_{s,i} = Theta_ss^{-1} e_1 / sqrt(e_1^T Theta_ss^{-1} e_1) (eq. L_col),
 * from an FP64 square-root-free Cholesky factorization (L D L^T) of Theta_ss.
 *
 *   pts        [n][dim] FP64 coordinates
 *   targets    [n_targets] int32 column ids
 *   pool_idx   [n_targets][pool_stride] int32 candidate ids
 *   pool_len   [n_targets] int32, 0 <= pool_len <= pool_stride <= csel_max_pool()
 *   k          0 <= k <= csel_max_select()
 *   precision  CSEL_FP64: everything in FP64.
 *              CSEL_MIXED: covariance evaluation and the left-looking GEMV of
 *              the selection in FP32; conditional variances/covariances,
 *              Theta_ss and its L D L^T factorization in FP64; candidates
 *              ranked by the FP32 value of the FP64 score cov^2 / var (equal
 *              values to the smaller pool slot), with or without top2_gap.
 * Outputs (per column c):
 *   sel_idx    [n_targets][k] selected ids in selection order, -1 padded
 *   factor_val [n_targets][k+1]: [0] = L_ii, [1+t] = entry of row sel_idx[t];
 *              0 in padded slots
 *   log_condvar[n_targets] log Theta_{ii | s_i \ i} (may be NULL); the sum
 *              over all columns minus log det Theta is 2 KL (eq. obj_chol)
 *   top2_gap   [n_targets][k] relative gap (s1 - s2)/s1 between the best and
 *              second-best scores at each step (the ranked scores: FP64, or
 *              FP32 in CSEL_MIXED), 1 with a single eligible candidate, NaN
 *              padded (may be NULL).  Asking for it changes no other output.
 *   status     [n_targets] per-column status (see above)
 */
int csel_select_and_factor(const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel,
                           int64_t n_targets, const int32_t *targets, const int32_t *pool_idx,
                           const int32_t *pool_len, int32_t pool_stride, int32_t k, int32_t precision,
                           int32_t *sel_idx, double *factor_val, double *log_condvar, float *top2_gap,
                           uint8_t *status, hipStream_t stream);

/*
 * csel_select_and_factor_sched -- csel_select_and_factor under an explicit
 * schedule, without the top2_gap output.  Same computation and results, bit
 * for bit, under every schedule; only the speed differs (chosen by a tuner).
 *
 *   col_list, col_count, max_cols  NULL/NULL: every column in its natural
 *              order (max_cols ignored); else the columns col_list[0 ..
 *              *col_count), as for csel_select_and_factor_list
 *   waves_per_column  1: one wavefront holds a column's whole pool (the
 *              schedule of csel_select_and_factor); or
 *              csel_select_waves_per_column(pool_stride) (2 for pools <= 128,
 *              4 up to 512): the pool split over that many wavefronts of a
 *              workgroup, which exchange each pick's argmax and winning row
 *              through LDS -- fewer registers per wavefront, so more of them
 *              resident (CSEL_EUNSUPPORTED for other values)
 */
int32_t csel_select_waves_per_column(int32_t pool_stride);
int csel_select_and_factor_sched(const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel,
                                 int64_t n_targets, const int32_t *targets, const int32_t *pool_idx,
                                 const int32_t *pool_len, int32_t pool_stride, int32_t k, int32_t precision,
                                 const int32_t *col_list, const int32_t *col_count, int64_t max_cols,
                                 int32_t waves_per_column, int32_t *sel_idx, double *factor_val, double *log_condvar,
                                 uint8_t *status, hipStream_t stream);

/*
 * csel_select_global -- greedy single-target selection with the nonzeros
 * allocated over the columns by global greedy selection (Sec. 5.4, eq.
 * global_obj): of a budget of off-diagonal nonzeros, each next one goes to
 * the column whose next greedy pick removes the largest fraction of its
 * target's conditional variance (the pick's squared conditional correlation,
 * a monotone image of its exact decrease of the KL divergence of eq.
 * obj_chol), equal fractions to the smaller column index; a column never
 * receives more than k_max or than its greedy selection finds.
 *
 * Inputs as csel_select_and_factor (k_max in place of k) plus
 *   budget     total off-diagonal nonzeros to allocate (>= 0; with more than
 *              all columns can take, every column gets its whole run)
 *   workspace  device scratch of csel_select_global_workspace_size(n_targets,
 *              k_max) bytes, caller-owned, no initialization
 * Outputs:
 *   k_alloc    [n_targets] nonzeros allocated to each column
 *   sel_idx    [n_targets][k_max] the first k_alloc greedy picks, -1 after
 *   factor_val [n_targets][k_max+1], log_condvar [n_targets] (may be NULL):
 *              the eq. L_col column on i and its allocated picks, laid out as
 *              for csel_select_and_factor
 *   gain       [n_targets][k_max] (may be NULL) the fraction of the target's
 *              conditional variance removed by each greedy step up to k_max
 *              (the allocation's keys), NaN past the column's last pick
 *   status     as for csel_select_and_factor (0 or 3)
 * The selection runs in its top-two form (FP64 score keys).
 */
int64_t csel_select_global_workspace_size(int64_t n_targets, int32_t k_max);
int csel_select_global(const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel, int64_t n_targets,
                       const int32_t *targets, const int32_t *pool_idx, const int32_t *pool_len, int32_t pool_stride,
                       int32_t k_max, int64_t budget, int32_t precision, void *workspace, int64_t workspace_bytes,
                       int32_t *k_alloc, int32_t *sel_idx, double *factor_val, double *log_condvar, double *gain,
                       uint8_t *status, hipStream_t stream);

/*
 * csel_aggregated_workspace_size -- bytes of device workspace that
 * csel_aggregated_select needs for these sizes (-1 with csel_last_error set if
 * the sizes are not supported).  The workspace holds the two partial Cholesky
 * factors of the groups in flight; its contents need no initialization and
 * are scratch after the call.
 */
int64_t csel_aggregated_workspace_size(int64_t n_groups, int32_t pool_stride, int32_t max_members, int32_t k,
                                       int32_t precision);

/* Largest aggregated pattern |s_g| = members + selected for which
 * csel_aggregated_select can build the member columns (status 5 beyond). */
int32_t csel_aggregated_max_block(void);

/*
 * csel_aggregated_select -- multi-target greedy selection for groups of
 * columns (supernodes) sharing one sparsity set, with the aggregated factor
 * columns and/or GP posterior variances.
 *
 * For group g with targets T = members[group_ptr[g] .. group_ptr[g+1]) and
 * candidates pool_idx[g*pool_stride + 0 .. pool_len[g]), k_g = min(k,
 * pool_len[g]) points are selected one at a time, each maximizing the
 * decrease of log det Theta_{TT | I} (D-optimal design, eq. greedy_mult):
 * log Theta_{jj | I, T} - log Theta_{jj | I}, computed as the score
 * 1 - var2_j / var1_j from two partial Cholesky factors -- one conditioned on
 * the targets first and then on the selected points, one on the selected
 * points only (Sec. 5.2; App. C.2).  Eligibility and ties as in
 * csel_select_and_factor (both conditional variances above 1e-12 times the
 * prior).
 *
 *   members      [sum m] int32 target ids, ascending within each group
 *                (with factor output, a group whose members are not strictly
 *                ascending gets status 3)
 *   group_ptr    [n_groups+1] int32 CSR offsets, 1 <= m_g <= max_members
 *   max_members  bound on every m_g (groups above it get status 3)
 *   pool_idx     [n_groups][pool_stride] int32 candidate ids, pool_len [n_groups]
 *   k            0 <= k <= 256; pool_stride + max_members <= 4096
 *   precision    CSEL_FP64, or CSEL_MIXED: FP64 conditional variances and
 *                factor columns; the covariance evaluations and GEMVs of the
 *                picks-only factor (var1) in FP32; those of the
 *                target-conditioned factor (var2) in FP32 for pools <= 512,
 *                groups <= 32, k <= 64 without post_var, in FP64 otherwise
 *   workspace    device scratch of csel_aggregated_workspace_size() bytes
 * Outputs:
 *   sel_idx      [n_groups][k] selected ids in selection order, -1 padded
 *   top2_gap     [n_groups][k] relative top-two score gap per step (may be NULL)
 *   group_logdet [n_groups] log det Theta_{TT | selected} tracked during the
 *                selection; with adjacent groups this is the group's KL term
 *                (eq. obj_mult) (may be NULL)
 *   post_var     [sum m] Theta_qq | selected for every target: the posterior
 *                variances of GP prediction at the targets given the selected
 *                training points (Alg. infer_select) (may be NULL; CSEL_FP64
 *                only, CSEL_EUNSUPPORTED with CSEL_MIXED; NaN for a group with
 *                status 4, left unwritten for status 3)
 *   factor_val   (may be NULL) aggregated factor columns: member q gets
 *                s_q = {j in sort(T u selected) : j >= q} and the eq. L_col
 *                column on s_q, computed for the whole group from one reverse
 *                Cholesky factorization of Theta over sort(T u selected) in
 *                FP64 (App. A.4, eq. L_precision).  Requires every pool id to
 *                exceed every member id of its group (status 4 otherwise).
 *                Member a (0-based within its group of m_g members) owns the
 *                slots [val_ptr[a], val_ptr[a+1]) of factor_rows (row ids,
 *                ascending) and factor_val, which must hold m_g - a + k_g
 *                entries; unused trailing slots get row -1, value 0.
 *   member_log_condvar [sum m] log Theta_{qq | s_q \ q} (with factor_val)
 *   status       [n_groups] per-group status: 0, 1 (stopped early), 2 (block
 *                not positive definite), 3 (bad input), 4 (pool precedes a
 *                member with factor output), 5 (pattern larger than
 *                csel_aggregated_max_block(); selection outputs are valid),
 *                6 (results lost: a barrier wait among the workgroups that
 *                share the group ran out; not expected in a complete launch)
 * Schedule: runs of at most 128 groups whose pool_stride + max_members
 * exceeds 256, without factor output (and in mixed precision outside the
 * register kernel's range: pools <= 512, groups <= 32, k <= 64), split each
 * group's rows over workgroups of 1024, 512 or 256 threads launched
 * cooperatively (all resident at once); other runs, or when the device
 * cannot hold that grid, give each group one workgroup.  The two schedules
 * give bit-identical results.
 */
int csel_aggregated_select(const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel, int64_t n_groups,
                           const int32_t *group_ptr, const int32_t *members, int32_t max_members,
                           const int32_t *pool_idx, const int32_t *pool_len, int32_t pool_stride, int32_t k,
                           int32_t precision, void *workspace, int64_t workspace_bytes, int32_t *sel_idx,
                           float *top2_gap, double *group_logdet, double *post_var, const int64_t *val_ptr,
                           int32_t *factor_rows, double *factor_val, double *member_log_condvar, uint8_t *status,
                           hipStream_t stream);

/*
 * csel_aggregated_select_sched -- csel_aggregated_select under an explicit
 * schedule, for a caller that chooses by timing (the package's tuner does):
 *   CSEL_AGG_AUTO        the rule csel_aggregated_select follows
 *   CSEL_AGG_ONE_GROUP   one workgroup per group, factor columns in a slab
 *   CSEL_AGG_REGISTER    the mixed register kernel (CSEL_MIXED, no post_var,
 *                        pool_stride <= 512, max_members <= 32, k <= 64)
 *   CSEL_AGG_SPLIT_256/512/1024  each group's rows over cooperatively launched
 *                        workgroups of that many threads (no factor output,
 *                        n_groups <= 1024, k <= 256, max_members <= 128)
 * One workgroup per group and the split schedules give bit-identical results
 * (the same expressions and summation orders); the register kernel evaluates
 * the target-conditioned factor in FP32 and can differ in near-tied picks.
 * Errors: CSEL_EUNSUPPORTED for a schedule outside its range, or when a split
 * schedule's workgroups cannot all be resident at once.
 */
int csel_aggregated_select_sched(const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel,
                                 int64_t n_groups, const int32_t *group_ptr, const int32_t *members,
                                 int32_t max_members, const int32_t *pool_idx, const int32_t *pool_len,
                                 int32_t pool_stride, int32_t k, int32_t precision, void *workspace,
                                 int64_t workspace_bytes, int32_t *sel_idx, float *top2_gap, double *group_logdet,
                                 double *post_var, const int64_t *val_ptr, int32_t *factor_rows, double *factor_val,
                                 double *member_log_condvar, uint8_t *status, int32_t schedule, hipStream_t stream);

/*
 * csel_reverse_maximin -- the reverse-maximin ordering of Sec. 2.2 (eq.
 * maximin, p = 1) on the GPU: the last position holds point 0, and each
 * earlier position the remaining point farthest from every point placed
 * after it (squared distances summed over the coordinates in order, products
 * and sums rounded separately; ties to the smaller id); the same ordering as
 * the host definition, bit for bit.
 *   pts          [n][dim] FP64 in id order, 1 <= dim <= 3
 *   workspace    device scratch of csel_reverse_maximin_workspace_size(n, dim)
 *                bytes
 *   order        [n] int32 out: order[pos] = the id placed at position pos
 *   ell          [n] FP64 out: ell[pos] = distance of that point to the
 *                points at later positions (+inf at position n-1)
 *   rounds       host int32 out (may be NULL): rounds the GPU needed
 * Several points are placed per round (a prefix of the remaining points by
 * decreasing distance that no earlier point of it would change); the host
 * launches the rounds in batches and reads a progress counter between them,
 * so the call returns after the stream has drained.
 * Errors: CSEL_EHIP if the rounds stop making progress (not expected).
 */
int64_t csel_reverse_maximin_workspace_size(int64_t n, int32_t dim);
int csel_reverse_maximin(const double *pts, int64_t n, int32_t dim, void *workspace, int64_t workspace_bytes,
                         int32_t *order, double *ell, int32_t *rounds, hipStream_t stream);

/*
 * csel_later_knn -- the later-ordered candidate pools of Sec. 4 on the GPU:
 * for every ordering position i (points in ordering-position order), the C
 * nearest points among positions i+1 .. n-1, ascending by squared distance
 * (summed over the coordinates in order, products and sums rounded
 * separately), then position; the same pools as the host definition, bit
 * for bit.
 *   pts          [n][dim] FP64, 1 <= dim <= 3
 *   C            0 <= C <= 2048
 *   workspace    device scratch of csel_later_knn_workspace_size(n, dim) bytes
 *   pool_idx     [n][C] int32 out, -1 padded
 *   pool_len     [n] int32 out: min(C, n-1-i); -1 (row all -1) only when more
 *                than 2048 later points tie at one distance around the C-th
 * Errors: CSEL_EUNSUPPORTED for C above 2048.
 */
int64_t csel_later_knn_workspace_size(int64_t n, int32_t dim);
int csel_later_knn(const double *pts, int64_t n, int32_t dim, int32_t C, void *workspace, int64_t workspace_bytes,
                   int32_t *pool_idx, int32_t *pool_len, hipStream_t stream);

/*
 * csel_partial_select -- partial (non-adjacent) aggregated selection, FP64
 * (Sec. 5.1 eq. chol_partial and eq. partial_kl; App. C.3).  As
 * csel_aggregated_select, but the candidates may lie between the group's
 * members: a selected point j joins the pattern of every member q < j (it
 * conditions only the members it follows), and the group term minimized is
 * sum_{q in T} log Theta_{qq | s_q \ q}, s_q = {j in T u S : j > q}, the log
 * determinant of the partially conditioned member covariance.  Each pick
 * maximizes its decrease: over the members j conditions, walking the
 * columns (selected and member points by decreasing id) with v = Theta_{jj |
 * columns before}, a member's variance falls by 1 - L_jc^2 / v (eq.
 * obj_partial) and then v -= L_jc^2 (eq. partial_induct); the score is
 * 1 - prod (1 - L_jc^2 / v), in [0, 1].  Eligible: v > 1e-12 times the prior
 * variance after the last column; ties to the smaller pool slot.  With every
 * candidate after every member this is csel_aggregated_select's selection.
 *
 *   members      [sum m] int32 member ids, strictly ascending within a group
 *   group_ptr    [n_groups+1]; 1 <= m_g <= max_members <= 32
 *   pool_idx     [n_groups][pool_stride] candidate ids (no member, no repeat),
 *                pool_len [n_groups]; pool_stride <= 512; k <= 32; every
 *                group needs m_g + min(k, pool_len) <= 64
 * Outputs: sel_idx, top2_gap (may be NULL), group_logdet (the group term
 * after the picks, may be NULL), status (0, 1 stopped early, 2 not positive
 * definite, 3 bad input: a member or pool id out of range, members not
 * strictly ascending, a pool id that is a member or repeats, or a size
 * above the limits), and, with factor_val, the member columns exactly as in
 * csel_aggregated_select (member a owns m_g - a + k_g slots at val_ptr;
 * eq. L_col on s_q = {j in sort(T u S) : j >= q}) and member_log_condvar,
 * whose sum over a group is its group term (eq. partial_kl).
 * Errors: CSEL_EUNSUPPORTED for sizes above the limits.
 */
int csel_partial_select(const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel, int64_t n_groups,
                        const int32_t *group_ptr, const int32_t *members, int32_t max_members,
                        const int32_t *pool_idx, const int32_t *pool_len, int32_t pool_stride, int32_t k,
                        int32_t *sel_idx, float *top2_gap, double *group_logdet, const int64_t *val_ptr,
                        int32_t *factor_rows, double *factor_val, double *member_log_condvar, uint8_t *status,
                        hipStream_t stream);

/*
 * csel_apply_factor -- product with a sparse lower-triangular factor L in CSC
 * form, the way the factor is used once built (L L^T ~ Theta^{-1}; e.g. as a
 * preconditioner, Sec. 6.3).
 *
 *   n          number of columns (= rows) of L
 *   col_ptr    [n+1] int64 offsets into row_idx / val
 *   row_idx    [nnz] int32 row of each entry; entries with a negative row (or
 *              a row >= n) are skipped, so the padded [T][k+1] layout of
 *              csel_select_and_factor can be passed with col_ptr[j] = j*(k+1)
 *   val        [nnz] FP64 values
 *   transpose  1: y = L^T x (per-column gather, deterministic)
 *              0: y = L x (per-column scatter with FP64 atomics; the order of
 *                 the additions, and so the last bits, may vary between runs)
 *   x, y       [n] FP64; must not alias
 */
int csel_apply_factor(int64_t n, const int64_t *col_ptr, const int32_t *row_idx, const double *val,
                      int32_t transpose, const double *x, double *y, hipStream_t stream);

/*
 * csel_kernel_matvec -- y = Theta x for the dense kernel matrix Theta of the
 * points (Matern kernel plus the nugget on the diagonal), matrix-free in
 * FP64: every entry is evaluated as it is used, O(n^2) work and O(n) memory.
 * Deterministic (partial sums over column chunks added in a fixed order).
 *
 *   x, y       [n] FP64, must not alias
 *   workspace  csel_kernel_matvec_workspace_size(n) bytes of device scratch
 */
int64_t csel_kernel_matvec_workspace_size(int64_t n);
int csel_kernel_matvec(const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel, const double *x,
                       double *y, void *workspace, int64_t workspace_bytes, hipStream_t stream);

/*
 * csel_pcg -- solve Theta x = y by the conjugate gradient preconditioned by
 * a sparse inverse-Cholesky factor L (L L^T ~ Theta^{-1}, so the
 * preconditioner is z = L (L^T r)), the use of the factor of Sec. 6.3.  The
 * points and every vector are in the factor's ordering.
 *
 *   l_col_ptr, l_row_idx, l_val     L in CSC form (as for csel_apply_factor);
 *                                   NULL for the plain conjugate gradient
 *   lt_col_ptr, lt_row_idx, lt_val  L^T in CSC form (csel_transpose_factor)
 *   y          [n] right-hand side
 *   x          [n] in: the initial guess; out: the solution
 *   rel_tol    stop when ||y - Theta x|| <= rel_tol ||y|| (the residual
 *              recurrence's norm), or after max_iter iterations
 *   iterations, rel_residual   HOST outputs: iterations taken, final
 *              relative residual norm
 *   workspace  csel_pcg_workspace_size(n) bytes of device scratch
 * Each iteration is one kernel matrix-vector product, two factor products
 * and three dot products on `stream`; the call synchronizes `stream` once
 * per iteration to read the residual norm.
 */
int64_t csel_pcg_workspace_size(int64_t n);
int csel_pcg(const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel, const int64_t *l_col_ptr,
             const int32_t *l_row_idx, const double *l_val, const int64_t *lt_col_ptr, const int32_t *lt_row_idx,
             const double *lt_val, const double *y, double *x, double rel_tol, int32_t max_iter, void *workspace,
             int64_t workspace_bytes, int32_t *iterations, double *rel_residual, hipStream_t stream);

/*
 * csel_transpose_factor -- the CSC form of L^T from the CSC form of L (that
 * is, L by rows), for y = L x as a deterministic gather: csel_apply_factor
 * with transpose = 1 on the result computes y = (L^T)^T x = L x with the
 * same per-column gather as y = L^T x, without the atomics of transpose = 0.
 * Build it once per factor.
 *
 *   n, col_ptr [n+1], row_idx, val   L as for csel_apply_factor, with
 *              0 <= col_ptr[j] <= col_ptr[j+1] and n_slots = col_ptr[n]
 *              stored slots (n < 2^31 - 1, n_slots < 2^31)
 *   t_col_ptr  [n+1] int64 out: column r of L^T (row r of L) is
 *              [t_col_ptr[r], t_col_ptr[r+1])
 *   t_row_idx, t_val  [n_slots] out: the column of L and the value of each
 *              entry, ascending column inside a row (a stable sort of the
 *              slots by row); slots with a row outside [0, n) are dropped,
 *              and the slots past t_col_ptr[n] get row -1 and value 0
 *   workspace  device memory of csel_transpose_factor_workspace_size(n,
 *              n_slots) bytes, caller-owned, not kept after the call's work
 */
int64_t csel_transpose_factor_workspace_size(int64_t n, int64_t n_slots);
int csel_transpose_factor(int64_t n, const int64_t *col_ptr, const int32_t *row_idx, const double *val,
                          int64_t n_slots, int64_t *t_col_ptr, int32_t *t_row_idx, double *t_val, void *workspace,
                          int64_t workspace_bytes, hipStream_t stream);

/*
 * csel_select_and_factor_list -- csel_select_and_factor restricted to the
 * columns col_list[0 .. *col_count) (device int32 list and count), e.g. the
 * fallback columns reported by csel_screen.  Array arguments are indexed by
 * column exactly as in csel_select_and_factor; only listed columns are
 * written.  max_cols bounds *col_count (the launch covers max_cols columns,
 * listed entries beyond *col_count are ignored), so the call needs no host
 * synchronization.
 */
int csel_select_and_factor_list(const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel,
                                int64_t n_targets, const int32_t *targets, const int32_t *pool_idx,
                                const int32_t *pool_len, int32_t pool_stride, int32_t k, int32_t precision,
                                const int32_t *col_list, const int32_t *col_count, int64_t max_cols,
                                int32_t *sel_idx, double *factor_val, double *log_condvar, float *top2_gap,
                                uint8_t *status, hipStream_t stream);

/*
 * Screened-selection plan.  A plan holds everything the learned-screened step
 * needs besides the caller's inputs and outputs -- the screen's kept lists,
 * flags, fallback list and count, the columns' processing order, the
 * schedules of the two selections (tuned on the plan's first step) and,
 * with CSEL_PLAN_GRAPH, the whole step captured as one HIP graph -- so the
 * step is a single call with no host synchronization after the first.
 * Device memory is allocated by csel_plan_create on the current device and
 * released by csel_plan_destroy; a step allocates nothing.  A plan serves one
 * problem shape (n_targets, pool_stride, keep, k, precision) on the device it
 * was created on, and may not be used by two threads at once.
 */
typedef struct csel_plan csel_plan;

enum { CSEL_PLAN_GRAPH = 1 };  /* replay the step from a captured HIP graph */

/*
 * csel_plan_create -- a plan for csel_screened_select over n_targets columns
 * with pools of up to pool_stride (<= csel_max_pool()) candidates, screened to
 * `keep` (1 <= keep <= pool_stride) before the greedy selection of
 * k (<= csel_max_select()) in `precision`.  Buffers: about
 * n_targets * (4 keep + 13) bytes plus the order's sort workspace.
 * *plan is NULL on failure (CSEL_ENOMEM when the buffers do not fit).
 */
int csel_plan_create(csel_plan **plan, int64_t n_targets, int32_t pool_stride, int32_t keep, int32_t k,
                     int32_t precision, uint32_t flags);

/* csel_plan_destroy -- waits for the device, then frees the plan (NULL ok). */
void csel_plan_destroy(csel_plan *plan);

/*
 * csel_plan_set_order -- the columns' processing order for the plan's steps:
 * the Morton order of the targets (csel_spatial_order), computed on `stream`
 * into the plan.  Without it the columns run in their natural order.  The
 * next step tunes the kept-pool schedule again.
 */
int csel_plan_set_order(csel_plan *plan, const double *pts, int64_t n, int32_t dim, const int32_t *targets,
                        hipStream_t stream);

/*
 * csel_screened_select -- one learned-screened step, the hot path of the
 * benchmark: per column (Sec. 3.1 on a pruned pool):
 *   1. csel_screen: features, MLP, the `keep` best candidates, fallback flag
 *      and the device-side fallback list (processing order from
 *      csel_plan_set_order, if set);
 *   2. csel_select_and_factor on the kept pools (natural or Morton column
 *      order, one or several waves per column: whichever the plan's first
 *      step timed fastest);
 *   3. csel_select_and_factor on the full pools of the fallback columns
 *      (csel_select_and_factor_list over the device-side list, its launch
 *      covering every column: no host read of the count).
 * Inputs and outputs are those of csel_screen and csel_select_and_factor for
 * the plan's shape (targets [n_targets], pool_idx [n_targets][pool_stride],
 * sel_idx [n_targets][k], factor_val [n_targets][k+1], log_condvar
 * [n_targets] (may be NULL), status [n_targets]); no top2_gap.  The plan's
 * first step (and the first after csel_plan_set_order) runs eagerly and
 * synchronizes `stream` to time the schedules; later steps enqueue
 * asynchronously.  With CSEL_PLAN_GRAPH later steps replay one captured HIP
 * graph, captured again whenever a pointer or scalar argument changes.
 */
int csel_screened_select(csel_plan *plan, const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel,
                         const int32_t *targets, const int32_t *pool_idx, const int32_t *pool_len,
                         const float *params, const uint16_t *params_bf16, float fallback_threshold,
                         int32_t *sel_idx, double *factor_val, double *log_condvar, uint8_t *status,
                         hipStream_t stream);

/*
 * csel_plan_info -- the plan's tuned schedules (host outputs, any may be
 * NULL): *kept_schedule for the kept-pool selection (-1 not yet tuned; bit 0
 * the Morton column order, else natural; bit 1 the multi-wave schedule of
 * csel_select_and_factor_sched, else one wave per column), *fallback_waves
 * for the fallback columns' launch, and tune_ms[6] the tuning step's times in
 * ms (kept pools under schedules 0-3, 0 where not timed; the fallback launch
 * under one wave and under the multi-wave schedule).
 */
int csel_plan_info(const csel_plan *plan, int32_t *kept_schedule, int32_t *fallback_waves, float *tune_ms);

/*
 * csel_plan_screen_outputs -- device-to-device copies, enqueued on `stream`,
 * of the last step's screen outputs held by the plan: kept_idx
 * [n_targets][keep], kept_len [n_targets], fallback [n_targets] (as in
 * csel_screen), fallback_list [n_targets] and fallback_count [1]; any
 * destination may be NULL.
 */
int csel_plan_screen_outputs(const csel_plan *plan, int32_t *kept_idx, int32_t *kept_len, uint8_t *fallback,
                             int32_t *fallback_list, int32_t *fallback_count, hipStream_t stream);

/*
 * Learned candidate screen (not part of the paper).  An MLP scores every
 * candidate of a column from 16 geometric features; the `keep` best are
 * kept, and the exact greedy selection of csel_select_and_factor runs on the
 * kept candidates.  The MLP is 16 -> 64 -> 64 -> 1 with ReLU, evaluated with
 * BF16 inputs, weights and hidden-layer activations on MFMA, FP32
 * accumulation and FP32 biases.  Parameters are one FP32 vector of
 * csel_mlp_num_params() values, W1[16][64], b1[64], W2[64][64], b2[64],
 * w3[64], b3, plus its BF16 copy (uint16 bit patterns, same indexing).
 *
 * Features of candidate j at pool slot s of target i (d = x_j - x_i, r = |d|,
 * slot 0 nearest): log(r/r_0), s/C, K(r)/variance, r/length_scale,
 * r_0/length_scale, cos(d, d_0), the smallest distance from x_j to one of the
 * 8 nearest candidates over r, the fraction of those 8 that are closer than
 * j within a 0.7-cosine cone, K(|x_j - x_{p0}|)/variance, the target-variance
 * decrease j would bring after the nearest candidate is selected (eq.
 * obj_gp), [s == 0], log(1+s)/log(1+C), and 4 zeros.
 */
int32_t csel_mlp_num_params(void);

/* Features [n_targets][pool_stride][16] (FP32) of every pool slot < pool_len. */
int csel_screen_features(const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel, int64_t n_targets,
                         const int32_t *targets, const int32_t *pool_idx, const int32_t *pool_len,
                         int32_t pool_stride, float *features, hipStream_t stream);

/*
 * csel_screen -- per column: features, MLP logits, the `keep` largest logits
 * (ties to the smaller slot), written as candidate ids in slot (distance)
 * order to kept_idx [n_targets][keep] (-1 padded), kept_len [n_targets].
 * Columns with pool_len <= keep keep their whole pool.  fallback[c] = 1 when
 * the dropped candidates' summed sigmoid(logit) (their expected number of
 * selections) exceeds fallback_threshold; such columns should be selected on
 * their full pool, and when fallback_list/fallback_count are given their
 * indices are appended there (count reset by this call; list order is not
 * deterministic).  fallback = 3 marks bad input (target, pool index or pool
 * length out of range): nothing is kept, and the column is appended to
 * fallback_list as well, so the full-pool selection reports it (status 3)
 * rather than the kept-pool selection answering for an empty pool.  logits [n_targets]
 * [pool_stride] is optional.  pool_stride <= 512.
 *
 * order, n_order (optional): the device int32 list order[0 .. n_order) of the
 * columns to process, in that order, e.g. csel_spatial_order's output or a
 * slice of it; results do not depend on the order.  A column absent from it
 * is not processed (its outputs are left as they were); entries outside
 * [0, n_targets) are skipped; a column listed twice is processed twice (its
 * fallback index is then appended twice).  n_order <= n_targets
 * (CSEL_EINVAL otherwise), so the fallback list -- n_targets entries -- never
 * receives more than it holds.  With order NULL, n_order is ignored and 0, 1,
 * ..., n_targets - 1 are processed.
 */
int csel_screen(const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel, int64_t n_targets,
                const int32_t *targets, const int32_t *pool_idx, const int32_t *pool_len, int32_t pool_stride,
                const float *params, const uint16_t *params_bf16, int32_t keep, float fallback_threshold,
                int32_t *kept_idx, int32_t *kept_len, uint8_t *fallback, float *logits, int32_t *fallback_list,
                int32_t *fallback_count, const int32_t *order, int64_t n_order, hipStream_t stream);

/*
 * csel_screen_groups -- the learned screen for multi-target groups (the
 * aggregated selection of Sec. 5 and GP prediction batches, Alg.
 * infer_select): prunes each group's candidate pool to the `keep`
 * candidates the MLP scores highest, before csel_aggregated_select runs on
 * the kept pools.  Not part of the paper.  One workgroup per group.
 *
 *   group_ptr [n_groups + 1], members [n_members]   CSR groups of 1..64
 *              member ids (as for csel_aggregated_select)
 *   pool_idx [n_groups][pool_stride] (pool_stride <= 2048), pool_len
 *              [n_groups]: candidates sorted by the distance to the nearest
 *              member, nearest first
 *   features   with r_q the distances of candidate j (slot s of C) to the m
 *              members, r1 <= r2 the two smallest (r2 = r1 when m = 1), rho
 *              the kernel correlation, l the length scale:
 *              log(r1_s / r1_0), s/C, rho(r1), r1/l, rho(r2), mean rho(r_q),
 *              mean rho(r_q)^2, mean r_q / l, m/64, [s == 0],
 *              log(1+s)/log(1+C), then zeros to 16; FP32, the MLP sees them
 *              in BF16
 *   MLP        as in csel_screen (same parameter layout; trained on group
 *              selections)
 *   keep, kept_idx [n_groups][keep], kept_len, fallback
 *              the `keep` largest logits (equal logits: the smaller slot
 *              first), kept in slot order, -1 padded; fallback 1 when the
 *              dropped candidates' summed sigmoid(logit) exceeds
 *              fallback_threshold,
 *              3 for a bad group (member range or id, pool length or id out
 *              of range; kept_len 0; a caller re-selects it on its full pool
 *              like a fallback group, where csel_aggregated_select reports it)
 *   logits     optional [n_groups][pool_stride]
 *   features   optional FP32 [n_groups][pool_stride][16]; with params NULL
 *              the call computes features only (keep and the outputs of the
 *              screen are then ignored and may be NULL; bad groups are
 *              skipped)
 */
int csel_screen_groups(const double *pts, int64_t n, int32_t dim, const csel_kernel *kernel, int64_t n_groups,
                       const int32_t *group_ptr, const int32_t *members, int64_t n_members,
                       const int32_t *pool_idx, const int32_t *pool_len, int32_t pool_stride,
                       const float *params, const uint16_t *params_bf16, int32_t keep, float fallback_threshold,
                       int32_t *kept_idx, int32_t *kept_len, uint8_t *fallback, float *logits, float *features,
                       hipStream_t stream);

/*
 * csel_spatial_order -- a processing order of the columns by the Morton
 * (Z-order) code of their target points: coordinates quantised over the
 * targets' bounding box (10 bits per coordinate in 3-D, 15 in 2-D, 30 in
 * 1-D), sorted stably, so equal codes keep increasing column order.
 * order[k] (device int32 [n_targets]) is the k-th column to process.  Not
 * part of the paper: a schedule under which the columns in flight together
 * have nearby targets, so their candidate pools overlap in cache.  Targets
 * out of [0, n) are placed as if at the origin of the box.
 *
 *   workspace  device memory of csel_spatial_order_workspace_size(n_targets)
 *              bytes, caller-owned, not kept after the call's work ends
 */
int64_t csel_spatial_order_workspace_size(int64_t n_targets);
int csel_spatial_order(const double *pts, int64_t n, int32_t dim, int64_t n_targets, const int32_t *targets,
                       void *workspace, int64_t workspace_bytes, int32_t *order, hipStream_t stream);

/* MLP logits [n_rows] of feature rows x [n_rows][16]. */
int csel_mlp_forward(const float *params, const uint16_t *params_bf16, const float *x, int64_t n_rows,
                     float *logits, hipStream_t stream);

/* Workspace bytes for csel_mlp_grad. */
int64_t csel_mlp_grad_workspace_size(int64_t n_rows);

/*
 * csel_mlp_grad -- mean weighted binary cross-entropy with logits over the
 * rows (weight pos_weight on label 1, 1 on label 0) and its gradient with
 * respect to the parameters: grad [csel_mlp_num_params() + 1], the last entry
 * being the summed (not averaged) weighted loss.  Forward as in csel_screen;
 * backward with BF16 MFMA operands and FP32 accumulation; per-wave partial
 * gradients are summed in a fixed order (deterministic).
 */
int csel_mlp_grad(const float *params, const uint16_t *params_bf16, const float *x, const uint8_t *labels,
                  int64_t n_rows, float pos_weight, void *workspace, int64_t workspace_bytes, float *grad,
                  hipStream_t stream);

/*
 * csel_mlp_grad_noalloc -- csel_mlp_grad for callers that cannot allocate
 * device memory: code under HIP graph capture, tight training loops, and
 * harnesses that forbid allocation.  Same inputs, outputs and results (bit
 * for bit) as csel_mlp_grad, without the workspace argument: the per-wave
 * partial gradients go to a buffer of about 5.4 MB that the library holds on
 * each GPU it runs on, from its first call there until the process ends.
 * The call allocates nothing (no hipMalloc, no allocating library routine).
 *
 *   n_rows     0 <= n_rows <= CSEL_MLP_GRAD_NOALLOC_MAX_ROWS; larger batches
 *              get CSEL_EUNSUPPORTED (use csel_mlp_grad)
 *   stream     must belong to the calling thread's current device
 *
 * The first call on a device looks the buffer up there (make it before a
 * graph capture begins); later calls only enqueue kernels.  Every call on a
 * device shares that device's buffer: calls that may overlap on one GPU
 * (other streams, other threads) race and must be ordered by the caller.
 */
#define CSEL_MLP_GRAD_NOALLOC_MAX_ROWS 65536
int csel_mlp_grad_noalloc(const float *params, const uint16_t *params_bf16, const float *x, const uint8_t *labels,
                          int64_t n_rows, float pos_weight, float *grad, hipStream_t stream);

/* One Adam step (Kingma & Ba) on the FP32 parameters, step counted from 1;
 * m and v are the FP32 moment buffers; refreshes the BF16 copy. */
int csel_mlp_adam(float *params, uint16_t *params_bf16, const float *grad, float *m, float *v, int32_t n_params,
                  float lr, float beta1, float beta2, float eps, int32_t step, hipStream_t stream);

/* BF16 copy (round to nearest even) of the FP32 parameters. */
int csel_mlp_to_bf16(const float *params, uint16_t *params_bf16, int32_t n_params, hipStream_t stream);

/*
 * csel_sum -- deterministic FP64 sum of x[0..n) into *out (device scalar).
 * Used for S = sum_i log Theta_{ii|s_i \ i}, the data term of the KL
 * (eq. obj_chol).  The summation order is fixed, so results are bitwise
 * reproducible for a given n.
 */
int csel_sum(const double *x, int64_t n, double *out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* CSEL_H */
