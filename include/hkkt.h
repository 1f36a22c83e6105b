/*
 * hkkt.h -- C ABI of the MI355X hybrid direct-iterative KKT solver.
 *
 * Method: Regev, Chiang, Darve, Petra, Saunders, Swirydowicz, Peles,
 * "A Hybrid Direct-Iterative Method for Solving KKT Linear Systems".
 *
 * The solver handles the 2x2 block KKT system of Sec. 3 (eq. linsys2x2, with
 * the inequality block already eliminated, m_d = 0) with a regularised (1,1)
 * block:
 *
 *     K z = r,   K = [ H_delta  J^T ]   H_delta = H + D_x + delta*I,
 *                    [ J        0   ]   z = (x, y),  r = (r1, r2).
 *
 * Following Sec. 4 (eqs. linsys2x2mod, eq:gamma, Schur1, Schur2) it assembles
 * H_gamma = H_delta + gamma*J^T J on a fixed pattern, factors it by supernodal
 * Cholesky (one symbolic analysis per pattern, Sec. 2 reuse list), and solves
 *     S y = J H_gamma^{-1} rhat - r2,  S = J H_gamma^{-1} J^T,  rhat = r1 + gamma J^T r2
 * by unpreconditioned CG, then H_gamma x = rhat - J^T y (Algorithm 1, solve
 * phase). FP64 iterative refinement on the full KKT residual follows; in mixed
 * precision the factor and the triangular solves run in FP32 and an FP64
 * refactor is taken when refinement stalls.
 *
 * Conventions for every entry point:
 *  - Indices are 0-based. Row pointers are int64, column indices int32.
 *  - tril(H): lower triangle of H as CSR (rows), columns sorted and unique
 *    within a row; the diagonal may be absent (it is added structurally).
 *  - J: m x n_x CSR, columns sorted and unique within a row.
 *  - Value arrays follow the pattern order given to hkkt_analyze. Batched
 *    value arrays are batch-major and contiguous: instance b starts at
 *    b*nnz (or b*n_x, b*m).
 *  - Buffers are owned by the caller. Pointer mode (hkkt_options) says whether
 *    value/vector pointers are host or device (device = on the context's
 *    device, e.g. a torch tensor's data_ptr()). Pattern arrays given to
 *    hkkt_analyze are always host pointers and are copied.
 *  - The context owns its device memory: the symbolic tables, the factor (per
 *    instance, L storage entries in the factor's precision), a packed copy of
 *    the entries below the diagonal of the supernodes the wavefront solves
 *    handle (written by every factorization; at most the L storage again),
 *    the contribution-block and solve workspaces, and, for the staged
 *    tree-traversal solves, a solve copy of the top levels' panels built at
 *    the first triangular solve after each factorization. It grows on demand
 *    and is freed by hkkt_destroy.
 *  - Work is enqueued on the stream given to hkkt_create; entry points return
 *    after their outputs are written (factor: after its one status read;
 *    solve: after x and y are written).
 *  - Return codes: 0 OK; positive = numerical outcome the caller may act on
 *    (1 NOT_SPD, 2 CG_BREAKDOWN, 3 NOT_CONVERGED); negative = usage or device
 *    error with a message in hkkt_last_error (-1 ARG, -2 PATTERN, -3 STATE,
 *    -4 DEVICE, -5 OOM).
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef HKKT_H
#define HKKT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HKKT_OK = 0,
    HKKT_NOT_SPD = 1,         /* Cholesky of H_gamma met a pivot <= 0 or not finite */
    HKKT_CG_BREAKDOWN = 2,    /* CG's quadratic form fell below the breakdown threshold (rank-deficient J) */
    HKKT_NOT_CONVERGED = 3,   /* CG or refinement did not reach the tolerances */
    HKKT_ERR_ARG = -1,
    HKKT_ERR_PATTERN = -2,
    HKKT_ERR_STATE = -3,
    HKKT_ERR_DEVICE = -4,
    HKKT_ERR_OOM = -5
};

enum { HKKT_FP64 = 0, HKKT_MIXED = 1 };
enum { HKKT_PTR_HOST = 0, HKKT_PTR_DEVICE = 1 };

typedef struct hkkt_ctx hkkt_ctx;

typedef struct {
    int precision;          /* HKKT_FP64 or HKKT_MIXED (FP32 factor + solves, FP64 refinement) */
    int pointer_mode;       /* HKKT_PTR_HOST or HKKT_PTR_DEVICE */
    double cg_tol;          /* relative CG residual, Sec. 5.1 uses 1e-12 */
    double cg_tol_mixed;    /* inner CG tolerance when the operator is FP32 (default 1e-5) */
    double kkt_tol;         /* target relative KKT residual ||r - K z||_2 / ||r||_2 */
    double quad_form_eps;   /* breakdown if p'q <= eps*||p||^2*(p0'q0/||p0||^2) (default 1e-14) */
    double delta2;          /* 0: report CG_BREAKDOWN; > 0: restart CG on S + delta2*I (Algorithm 1);
                               either way a breakdown ends the solve after that pass (status 0 or 3
                               with delta2 > 0, 2 without) */
    int max_cg;             /* <= 0: min(m, 1000) */
    int max_refine;         /* refinement passes after the first (default 10) */
    int ordering;           /* 0 = own approximate minimum degree (Sec. 5.3), 1 = natural,
                               2 = nested dissection (level-structure bisection, AMD on small parts) */
    int relax;              /* supernode amalgamation: 0 none (fundamental), 1 default, 2 more */
    int deterministic;      /* 1: forward solves pull children's update vectors in a fixed order
                               (bitwise reproducible); 0: right-looking FP atomics (faster) */
    int mixed_check;        /* mixed precision: 1 applies each FP32 factor M once to a fixed probe
                               vector v and refactors in FP64 at factor time when
                               ||v - H_gamma M^{-1} v|| / ||v|| > mixed_check_tol; 0 (default):
                               only the stall test of the solve decides (measured faster on the
                               benchmark: the first FP32 pass still warms the FP64 start) */
    double mixed_check_tol; /* default 0.5 */
    int autotune_cache;     /* 1 (default): hkkt_autotune reuses the choice it made earlier in
                               this process for the same pattern (hash of the analysed pattern,
                               group layout and given order), precision and batch size instead
                               of timing again; 0: always time */
    int scaling;            /* 1: symmetrized Ruiz scaling of K (Sec. 4.1; ten sweeps d_i /= sqrt(max_j
                               |(D K D)_ij|)): the factorization and the hybrid passes work on D K D
                               (delta folded into its diagonal, gamma acting on the scaled J, i.e.
                               gamma * d_y^2 per J row), refinement on K's own residual; the factor
                               (hkkt_get_factor) and hkkt_hsolve are then those of the scaled
                               system. 0 (default): none */
    int flow_live;          /* applications of H_gamma^{-1} to at most this many instances (the CG
                               tail) run as one dataflow launch (each supernode task waits only for
                               its children / parent) instead of one launch per level; 0 = never.
                               Needs deterministic = 0 and every supernode within 128 rows.
                               Default 0: measured no faster than the level launches for one
                               live instance and slower for more (each task's agent-scope
                               release and acquire cost about as much as a launch) */
    int refine_inexact;     /* 1: refinement passes after the first stop CG at the relative residual
                               max(cg tolerance, min(1e-2, 0.1 * kkt_tol / RR)) of their instance
                               (the accuracy the correction needs to take RR below kkt_tol with a
                               tenfold margin); the first pass keeps the CG tolerance. 0 (default):
                               every pass at the CG tolerance */
    double mixed_pivot_tol; /* mixed precision: an FP32 factor whose smallest ratio of pivot L_jj^2
                               to the assembled FP64 diagonal a_jj of H_gamma is below this is
                               replaced by an FP64 factor at factor time: the FP32 success does not
                               show that H_gamma is positive definite (Algorithm 1's test), and a
                               pivot that kept fewer than about 12 of its 24 bits cannot drive
                               refinement to 1e-10 in fewer passes than an FP64 factor needs.
                               0 turns the test off (default 2^-12) */
} hkkt_options;

typedef struct {
    int status;             /* per instance, codes as above */
    int cg_iters;           /* total CG iterations over all passes */
    int passes;             /* hybrid passes (1 + refinement steps) */
    int fp64_fallback;      /* 1 if the instance was refactored in FP64 */
    int cg_iters_fp64;      /* of cg_iters, those run on an FP64 factor (all of them in FP64
                               precision; a mixed solve's after its fallback) */
    int passes_fp64;        /* of passes, those run on an FP64 factor */
    double rr;              /* ||r - K z||_2 / ||r||_2, FP64 on the device */
    double be;              /* ||r - K z||_2 / (||K||_inf ||z||_2 + ||r||_2), Sec. 5.1 */
    double floor;           /* 2^-53 * || |K||z| + |r| ||_2 / ||r||_2 */
    int64_t fail_col;       /* first failing pivot (original index) or -1 */
} hkkt_info;

/* Defaults: FP64, host pointers, cg_tol 1e-12, cg_tol_mixed 1e-5,
 * kkt_tol 1e-10, quad_form_eps 1e-14, delta2 0, max_cg 0, max_refine 10,
 * ordering 0, relax 1, deterministic 0, mixed_check 0, mixed_check_tol 0.5,
 * autotune_cache 1, scaling 0, flow_live 0, refine_inexact 0, mixed_pivot_tol 2^-12. */
void hkkt_default_options(hkkt_options *opt);

/* Create a context bound to the current HIP device and the given stream
 * (NULL = the null stream). Returns 0 or a negative code. */
int hkkt_create(hkkt_ctx **ctx, const hkkt_options *opt, void *hip_stream);
void hkkt_destroy(hkkt_ctx *ctx);
const char *hkkt_last_error(const hkkt_ctx *ctx);

/* Symbolic analysis, once per pattern (Sec. 2: ordering and symbolic
 * factorization are needed once per sequence; Sec. 5.3: AMD ordering).
 * Builds the pattern of H_gamma = tril(H) U diag U tril(J^T J), orders it
 * (own AMD, or `perm` if non-NULL: perm[k] = original index of the k-th
 * pivot), computes the elimination tree, supernodes, the assembly map and the
 * level schedules, and uploads them. Host pointers; copied. Errors: -2 on a
 * malformed pattern (unsorted/duplicate/out-of-range index, bad row pointers),
 * -1 if n_x < 1 or m < 0. */
int hkkt_analyze(hkkt_ctx *ctx, int64_t n_x, int64_t m,
                 const int64_t *H_rowptr, const int32_t *H_col,
                 const int64_t *J_rowptr, const int32_t *J_col,
                 const int32_t *perm);

/* Uneven batch in one launch: G independent KKT systems of different sizes
 * and patterns ("members") analysed together as one block-diagonal system,
 * so that every factor and solve kernel covers all of them (the Sec. 2
 * reuse list then holds per group). Member k owns the variables
 * [x_off[k], x_off[k+1]) and the J rows [y_off[k], y_off[k+1]) of the
 * combined pattern given as for hkkt_analyze (x_off[0] = y_off[0] = 0,
 * x_off[G] = n_x, y_off[G] = m; every member has at least one variable and
 * may have no J rows). Host arrays of G+1 entries; copied. Each member keeps
 * its own elimination range (own AMD order restricted to the member).
 * After it, hkkt_factor_batch / hkkt_solve_batch / hkkt_hsolve take the
 * combined value and vector arrays per batch entry, while every per-system
 * scalar and result is per (entry b, member k) at index b*G + k: delta,
 * gamma, status, fail_col (combined original index), info, and the index of
 * hkkt_inertia. Each member runs its own CG, refinement and FP64 fallback
 * (Algorithm 1 per member). hkkt_factor / hkkt_solve need G = 1.
 * Errors: -1 if G is not in [1, 65535], offsets missing or not increasing; -2 if an entry of
 * tril(H) or J couples two members, or as for hkkt_analyze. */
int hkkt_analyze_group(hkkt_ctx *ctx, int G, const int64_t *x_off, const int64_t *y_off,
                       int64_t n_x, int64_t m,
                       const int64_t *H_rowptr, const int32_t *H_col,
                       const int64_t *J_rowptr, const int32_t *J_col);

/* Autotuner (run once per pattern, after hkkt_analyze or
 * hkkt_analyze_group): times candidate schedules on the given values and
 * keeps the fastest. Candidates: supernode amalgamation relax in {0, 1, 2}
 * (supernode shapes: fewer, wider supernodes and fewer levels against more
 * stored zeros) x seven triangular-solve schedules: no tree kernel, then for
 * tree widths 8, 32, 128 (the top levels of at most that many supernodes
 * run in one tree-traversal launch) the staged tree kernel (right-hand side,
 * schedule and panels in LDS, where they fit) and the global-memory one.
 * Cost per candidate (milliseconds, host clock around synchronised work):
 * with right-hand sides r1, r2 (as for hkkt_solve_batch; r2 may be NULL when
 * m = 0), one hkkt_factor_batch plus one hkkt_solve_batch of the nb
 * instances, the faster of two such runs; with r1 = NULL a proxy: one factorization + one application of
 * H_gamma^{-1} to all instances + four applications to a list of min(nb, 8)
 * instances (the late CG iterations run on few instances). The chosen relax
 * is written to the context's options and the pattern is re-analysed with
 * it; choice[0] = relax, choice[1] = tree width, choice[2] = 1 for the
 * staged tree kernel. cost_ms (may be NULL) gets up to max_cost candidate
 * costs, relax-major, in the schedule order above (21 in all). Values as for
 * hkkt_factor_batch. The context is left analysed and not factored: call
 * hkkt_factor_batch next. Returns 0 or a negative code (-3 if not
 * analysed; a failed trial returns its code, e.g. -1 when r1 is given and
 * r2 is NULL while m > 0). On any failure the
 * context's schedule and profiling state are restored (the context is then
 * analysed with its previous relax and not factored). With autotune_cache
 * set, a choice already made for the same key is applied without timing
 * (cost_ms entries are then NaN). */
int hkkt_autotune(hkkt_ctx *ctx, int nb, const double *H_val, const double *D_x,
                  const double *J_val, const double *delta, const double *gamma,
                  const double *r1, const double *r2,
                  int32_t choice[3], double *cost_ms, int max_cost);

/* The context's current schedule, choice = (relax, tree width, staged tree
 * kernel) as hkkt_autotune reports it; -3 if not analysed. */
int hkkt_get_schedule(const hkkt_ctx *ctx, int32_t choice[3]);

/* Set the schedule (e.g. one the autotuner chose in an earlier run): relax in
 * {0, 1, 2}, tree width >= 0 (0 = no tree kernel), staged in {0, 1}. A
 * changed relax re-analyses the pattern and the context must be factored
 * again. -1 on values out of range, -3 if not analysed. */
int hkkt_set_schedule(hkkt_ctx *ctx, const int32_t choice[3]);

/* Numeric factorization of nb instances that share the analysed pattern
 * (Sec. 2: once per matrix; Algorithm 1's Cholesky attempt on H_gamma).
 * H_val [nb][nnz(tril H)], D_x [nb][n_x], J_val [nb][nnz(J)], delta [nb],
 * gamma [nb] (always host arrays for delta and gamma). status[b] (host, may
 * be NULL) gets 0 or HKKT_NOT_SPD; fail_col[b] (host, may be NULL) gets the
 * original index of the first failing pivot in elimination order, or -1.
 * The values are copied; the caller may reuse its buffers after return.
 * Returns 0 if every instance factored, 1 if any is NOT_SPD, negative on
 * error (-3 if not analysed). */
int hkkt_factor_batch(hkkt_ctx *ctx, int nb, const double *H_val, const double *D_x,
                      const double *J_val, const double *delta, const double *gamma,
                      int *status, int64_t *fail_col);

/* Algorithm 1's regularization of the (1,1) block around the Cholesky
 * attempt (Sec. 4.1), per (instance, member): factor with delta; while the
 * factorization fails and delta1 <= delta_max / 2, retry with delta + delta1,
 * where the first retry takes delta1 = delta_min[i] and every later one
 * doubles delta_min[i] and takes delta1 = delta_min[i]. delta_min (host,
 * [nb*G], every entry > 0) is in/out: it carries the last value tried into
 * the next matrix of a sequence (the listing's in-place update of
 * delta_min). delta1 (host, [nb*G]) gets the regularization used (0 when the
 * first attempt succeeded); status/fail_col as for hkkt_factor_batch, of the
 * last attempt (NOT_SPD left = Algorithm 1's fail-safe branch: the caller's
 * LDL^T or a return to the optimizer). The context then holds the factor of
 * H_gamma + (delta + delta1) I, and hkkt_solve_batch solves the perturbed
 * system K with delta + delta1 in its (1,1) block, as Algorithm 1 does. Each
 * retry refactors the whole batch (instances that succeeded get the same
 * factor again). Other arguments as for hkkt_factor_batch. Returns as
 * hkkt_factor_batch for the last attempt; -1 if delta_min <= 0 or
 * delta_max < 0. */
int hkkt_factor_regularized(hkkt_ctx *ctx, int nb, const double *H_val, const double *D_x,
                            const double *J_val, const double *delta, const double *gamma,
                            double *delta_min, double delta_max, double *delta1,
                            int *status, int64_t *fail_col);

/* The gamma heuristic of Sec. 3 (Golub and Greif): gamma = ||Htilde|| /
 * ||J||^2 per (instance, member), with Htilde = H + D_x + delta I and the
 * infinity norm standing in for the 2-norm (as Sec. 5.1 does for ||K||);
 * 0 when J is empty or zero. Values as for hkkt_factor_batch (no gamma);
 * gamma_out host [nb*G]. It loads the values into the context's batch on
 * the device, so the current factorization is dropped (factor again before
 * solving). Returns 0, or -3 if not analysed. */
int hkkt_gamma_heuristic(hkkt_ctx *ctx, int nb, const double *H_val, const double *D_x,
                         const double *J_val, const double *delta, double *gamma_out);

/* ---- the full 4x4 system of Sec. 3 (eq. linsys4x4) ------------------------
 *   K4 = [ H + D_x + delta I   0     J^T   J_d^T ]   z = (dx, ds, dy, dyd)
 *        [ 0                   D_s   0     -I    ]   r = (rx~, rs, ry, ryd)
 *        [ J                   0     0     0     ]
 *        [ J_d                 -I    0     0     ]
 * solved through the reduction of Sec. 3: ds = J_d dx - ryd, dyd = D_s ds - rs
 * leave the 2x2 system (eq. linsys2x2) with Htilde = H + D_x +
 * J_d^T D_s J_d and r_x = rx~ + J_d^T (D_s ryd + rs), which the hybrid
 * method solves (all the 2x2 options apply: precision, scaling, ...).
 *
 * hkkt_analyze4: patterns as for hkkt_analyze plus J_d (m_d x n_x CSR, host,
 * copied); the context is analysed for the 2x2 system on the pattern
 * tril(H) U tril(J_d^T J_d) (single system, no group). Errors as for
 * hkkt_analyze. A later hkkt_analyze / hkkt_analyze_group drops the 4x4
 * layer. */
int hkkt_analyze4(hkkt_ctx *ctx, int64_t n_x, int64_t m, int64_t m_d,
                  const int64_t *H_rowptr, const int32_t *H_col,
                  const int64_t *J_rowptr, const int32_t *J_col,
                  const int64_t *Jd_rowptr, const int32_t *Jd_col, const int32_t *perm);

/* Factor nb instances: H_val, D_x, J_val as for hkkt_factor_batch, Jd_val
 * [nb][nnz(J_d)], D_s [nb][m_d] (pointer mode), delta, gamma [nb] host.
 * Htilde's H part H + J_d^T D_s J_d is formed on the device on the combined
 * pattern (fixed summation order), then factored as hkkt_factor_batch does.
 * Returns as hkkt_factor_batch; -3 without hkkt_analyze4. */
int hkkt_factor4_batch(hkkt_ctx *ctx, int nb, const double *H_val, const double *D_x,
                       const double *J_val, const double *Jd_val, const double *D_s,
                       const double *delta, const double *gamma, int *status, int64_t *fail_col);

/* Solve K4 z = r for the factored instances: rx [nb][n_x], rs [nb][m_d],
 * ry [nb][m], ryd [nb][m_d] in, dx, ds, dy, dyd out (pointer mode). Each
 * step forms the 4x4 residual g = r - K4 z (plain FP64), reduces it to the
 * 2x2 right-hand side, solves the 2x2 system (with its own refinement),
 * recovers e_s = J_d e_x - g_yd, e_yd = D_s e_s - g_s and adds e to z, while
 * RR4 = ||g||/||r|| > kkt_tol and halves (at most max_refine + 1 steps). info
 * per instance: status, cg_iters (total), passes (4x4 steps), fp64_fallback,
 * rr and be on K4 (Sec. 5.1, ||K4||_inf), floor NaN (not computed for K4).
 * Returns the largest status or a negative code (-3 without factor4). */
int hkkt_solve4_batch(hkkt_ctx *ctx, int nb, const double *rx, const double *rs, const double *ry,
                      const double *ryd, double *dx, double *ds, double *dy, double *dyd,
                      hkkt_info *info);

/* Single-instance form of hkkt_factor_batch. */
int hkkt_factor(hkkt_ctx *ctx, const double *H_val, const double *D_x, const double *J_val,
                double delta, double gamma, int64_t *fail_col);

/* Solve K z = r for the nb instances of the last factorization (Algorithm 1
 * solve phase: rhat, w = H_gamma^{-1} rhat, CG on eq. Schur1, x from eq.
 * Schur2; then refinement to kkt_tol). r1 [nb][n_x], r2 [nb][m] in; x
 * [nb][n_x], y [nb][m] out; info [nb] (host, may be NULL; nb*G entries for
 * a group, see hkkt_analyze_group). nb must equal the last factorization's
 * nb. Returns the largest per-instance status (0 if all
 * converged), or negative on error (-3 if not factored successfully). */
int hkkt_solve_batch(hkkt_ctx *ctx, int nb, const double *r1, const double *r2,
                     double *x, double *y, hkkt_info *info);

int hkkt_solve(hkkt_ctx *ctx, const double *r1, const double *r2, double *x, double *y,
               hkkt_info *info);

/* Inertia (positive, negative, zero eigenvalue counts) of K for instance b
 * after a successful factor and solve (Sec. 4.2, Theorem 3: a successful
 * Cholesky of H_gamma gives n_x positive; with full-rank J the Schur
 * complement adds m negative). Returns 0 with (n_x, m, 0) when CG did not
 * break down. After a breakdown (J rank-deficient or nearly so) K has at
 * least one zero eigenvalue but the count is not known: returns
 * HKKT_CG_BREAKDOWN with out = (n_x, -1, -1) (n_x positive is still exact;
 * the other m are negative or zero). Returns -3 if no successful
 * factor+solve precedes it. */
int hkkt_inertia(const hkkt_ctx *ctx, int b, int64_t out[3]);

/* ---- host-only symbolic analysis handle (no GPU needed) ------------------
 * The same analysis hkkt_analyze runs, exposed for inspection and tests.
 * Arguments as for hkkt_analyze; ordering/relax as in hkkt_options. The
 * error message (if err is non-NULL) is written into err[errlen]. */
typedef struct hkkt_symbolic hkkt_symbolic;
int hkkt_symbolic_create(hkkt_symbolic **out, int64_t n_x, int64_t m,
                         const int64_t *H_rowptr, const int32_t *H_col,
                         const int64_t *J_rowptr, const int32_t *J_col,
                         const int32_t *perm, int ordering, int relax, char *err, int errlen);
/* Group form (members as for hkkt_analyze_group; perm may be NULL; a given
 * perm is regrouped by member, keeping its order within each member). */
int hkkt_symbolic_create_group(hkkt_symbolic **out, int G, const int64_t *x_off, const int64_t *y_off,
                               int64_t n_x, int64_t m,
                               const int64_t *H_rowptr, const int32_t *H_col,
                               const int64_t *J_rowptr, const int32_t *J_col,
                               const int32_t *perm, int ordering, int relax, char *err, int errlen);
void hkkt_symbolic_destroy(hkkt_symbolic *sym);

/* The analysis owned by a context (valid until the next hkkt_analyze). */
const hkkt_symbolic *hkkt_get_symbolic(const hkkt_ctx *ctx);

/* Symbolic statistics (host ints): stats[0] n_x, [1] m, [2] nnz(tril
 * H_gamma), [3] nnz(L) (structural), [4] L storage entries (supernodal
 * panels), [5] supernodes, [6] factor levels, [7] sum of c_j^2 over columns
 * (factor flop proxy), [8] max supernode width, [9] max supernode rows,
 * [10] contribution-block workspace entries per instance (ranges reused
 * across lifetimes), [11] etree height, [12] update
 * vector entries, [13] nnz(J). */
int hkkt_symbolic_stats(const hkkt_symbolic *sym, int64_t stats[16]);

/* Contribution-block workspace offsets (entries): cb_off[s] for supernode
 * s, cb_off[ns] = workspace size per instance (stats[10]). Blocks share
 * ranges when their lifetimes (from the supernode's level to its parent's)
 * do not overlap. */
int hkkt_symbolic_cb_offsets(const hkkt_symbolic *sym, int64_t *cb_off);

/* Final elimination order: perm[k] = original index of pivot k. */
int hkkt_symbolic_perm(const hkkt_symbolic *sym, int32_t *perm);

/* Supernode partition: sn_first [ns+1], sn_rowptr [ns+1], sn_rows
 * [sn_rowptr[ns]], sn_parent [ns], level_ptr [nlevels+1], level_sn [ns].
 * Any pointer may be NULL. */
int hkkt_symbolic_supernodes(const hkkt_symbolic *sym, int32_t *sn_first, int64_t *sn_rowptr,
                             int32_t *sn_rows, int32_t *sn_parent, int32_t *level_ptr,
                             int32_t *level_sn);

/* Copy the factor of batch entry b (for a group: the block-diagonal factor
 * of all members) into CSC form in the permuted order
 * (colptr [n_x+1], rowind, val [nnz(L)] in FP64), for parity tests. */
int hkkt_get_factor(hkkt_ctx *ctx, int b, int64_t *colptr, int32_t *rowind, double *val);

/* Apply H_gamma^{-1} (forward + backward supernodal triangular solves) of
 * instance set [0, nb) to b, in the original order: x = H_gamma^{-1} b.
 * Vectors [nb][n_x], per pointer mode. For parity tests. In mixed precision
 * the factor applied is the one the solve uses: FP32, or FP64 for the
 * instances the factorization sent to FP64 factors (their FP32
 * factorization stops at the first pivot below mixed_pivot_tol). */
int hkkt_hsolve(hkkt_ctx *ctx, int nb, const double *b, double *x);

/* Allocation-free form of hkkt_hsolve, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same triangular-solve kernels, with their
 * working vectors (the permuted right-hand side, the solve vector and, with
 * deterministic = 1, the update vectors) in a fixed device array of the
 * library (64 MiB per GPU, set up by hkkt_create and held until the process
 * ends) instead of library-allocated buffers. Needs pointer_mode =
 * HKKT_PTR_DEVICE: b [nb][n_x] and x [nb][n_x] are device pointers in the
 * original order, nb equal to the last factorization's. It allocates, frees
 * and synchronises nothing: the work is enqueued on the context's stream and
 * x is written when the stream reaches it. It reads the factor and its packed
 * solve copy, both written by the factorization. The staged tree kernel's panel
 * copy is used only if an earlier hkkt_solve/hkkt_hsolve after the last
 * factorization built it; otherwise the levels it would cover run in the
 * global-memory tree kernel (same solution up to rounding). Per-kernel
 * profiling is suspended during the call. Returns -1 for host pointer mode
 * or when 8*nb*n_x + (4 or 8)*nb*n_x (+ the update vectors) exceeds 64 MiB
 * (each part rounded up to 256 bytes), -3 if not factored, nb differs, or
 * (mixed precision) the factorization sent instances to FP64 factors: this
 * form applies the FP32 factor only. Every call on one GPU shares that
 * GPU's array: calls that overlap in time
 * on one GPU (other contexts or streams) race and must be serialised by the
 * caller; the array keeps the last call's contents, and every entry a call
 * reads is written by it first. */
int hkkt_hsolve_noalloc(hkkt_ctx *ctx, int nb, const double *b, double *x);

/* Time spent in the phases of the last calls (milliseconds, host clock
 * around stream-synchronised phases): [0] analyze, [1] assemble+factor,
 * [2] solve, [3] fp64 fallback. */
int hkkt_timings(const hkkt_ctx *ctx, double ms[8]);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * each launch, between hkkt_profile_begin and hkkt_profile_end. The end call
 * synchronises the stream and returns, per kernel class, the summed
 * launch durations ms[k] (milliseconds) and launch counts launches[k]
 * (arrays of HKKT_NPROF; either may be NULL). Classes: 0 assembly,
 * 1 LDS fronts, 2 large fronts (blocked), 3 forward solve (per-level
 * wavefront kernel), 4 backward solve (per-level wavefront kernel), 5 J^T
 * SpMV, 6 J SpMV, 7 CG vector updates, 8 CG scalars, 9 KKT residual,
 * 10 other, 11 triangular solves of very wide/tall supernodes, 12 both
 * triangular solves over the thin top levels of the tree (one launch, one
 * work-group per instance), 13 the same with the top levels' working set
 * staged in LDS, 14 both triangular solves over all levels as one dataflow
 * launch. */
#define HKKT_NPROF 15
int hkkt_profile_begin(hkkt_ctx *ctx);
/* Which launches hkkt_profile_begin/end record (an event pair on the
 * stream costs about as much as a short kernel): bit k of class_mask
 * selects class k, and of the selected classes only every `every`-th launch
 * of each class is recorded (the first one included); launches[] of
 * hkkt_profile_end then counts recorded launches. Default: all classes,
 * every launch. -1 if every < 1. */
int hkkt_profile_select(hkkt_ctx *ctx, unsigned class_mask, int every);
/* Which batches' launches hkkt_profile_begin/end record: -1 (default) all;
 * HKKT_FP64 or HKKT_MIXED only the work on factors of that precision (a
 * mixed-precision solver's FP64 fallback batches count as HKKT_FP64; the
 * FP64 completion of its factor-time fallbacks too). Kernels of one class
 * differ in element size between the two, so per-launch bytes do too.
 * -1 on any other value. */
int hkkt_profile_precision(hkkt_ctx *ctx, int precision);
int hkkt_profile_end(hkkt_ctx *ctx, double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif
