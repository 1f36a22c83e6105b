/*
 * oracle.c -- plain, slow, obviously correct FP64 CPU reference for the
 * hybrid direct-iterative KKT solve (Regev et al., "A Hybrid Direct-Iterative
 * Method for Solving KKT Linear Systems").
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library may link, call or
 * execute this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it. It shares no code with the GPU library.
 *
 * What it computes (Sec. 3 eq. linsys2x2 with m_d = 0, Sec. 4):
 *   K = [H + D_x + delta*I, J^T; J, 0],  K z = r,  z = (x, y), r = (r1, r2).
 *   H_gamma = H + D_x + delta*I + gamma*J^T J          (eq. eq:gamma)
 *   rhat    = r1 + gamma*J^T r2                        (eq. linsys2x2mod)
 *   S y     = J H_gamma^{-1} rhat - r2,  S = J H_gamma^{-1} J^T   (eq. Schur1)
 *   H_gamma x = rhat - J^T y                           (eq. Schur2)
 * solved as in Algorithm 1 (solve phase): w = H_gamma^{-1} rhat, CG on S,
 * then the primal recovery; followed by FP64 iterative refinement on the full
 * KKT residual, with the metrics of Sec. 5.1 (RR and BE with ||K||_inf).
 *
 * Every step is the textbook form: triplet assembly with sorted duplicate
 * summation, exact minimum degree on the explicit elimination graph,
 * left-looking column Cholesky (George & Liu), column-oriented forward and
 * dot-form backward substitution, unpreconditioned CG.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *  - CG starts from y = 0 and stops when ||res||_2 <= cg_tol * ||b||_2
 *    (Sec. 5.1: relative residual tolerance 1e-12), or after max_cg steps.
 *  - Algorithm 1's breakdown test on the quadratic form has no threshold in
 *    the paper: breakdown when p'q <= qf_eps*||p||^2*(p0'q0/||p0||^2).
 *  - refinement: while RR > kkt_tol and steps < max_refine: solve K e = res by
 *    the same hybrid steps, z += e, recompute res = r - K z.
 *  - inertia of K after a successful Cholesky of H_gamma and CG without
 *    breakdown: (n_x, m, 0) (Sec. 4.2, Theorem 3; congruence + Haynsworth).
 *    After a breakdown only the n_x positive eigenvalues are determined: the
 *    other m split between negative and at least one zero (reported as -1).
 *  - the KKT residual r - K z that RR, BE and refinement use is evaluated
 *    with compensated dot products (error-free TwoProduct by FMA and TwoSum,
 *    Ogita, Rump and Oishi 2005, "Accurate sum and dot product", algorithm
 *    Dot2), every product of a stored value with an entry of z a term of its
 *    own (K's diagonal is H_ii + D_i + delta, three terms), so the residual
 *    is as accurate as if computed in twice the working precision: the plain
 *    FP64 sum has an error near u * || |K||z| + |r| || (the "floor"), which
 *    on these inputs can exceed the 1e-10 target itself.
 *  - the best RR any FP64 z can be expected to reach is that of the
 *    correctly rounded exact solution; orc_refine_dd computes it by
 *    refinement with z held as an unevaluated sum of two doubles.
 *
 * Build with -ffp-contract=off: the error-free transformations need every
 * product and sum rounded on its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t i64;
typedef int32_t i32;

/* ------------------------------------------------------------------ */
/* system                                                              */
/* ------------------------------------------------------------------ */

typedef struct {
    i64 n, m;
    /* tril(H) CSR (rows), J CSR */
    i64 *Hp; i32 *Hi; double *Hx;
    i64 *Jp; i32 *Ji; double *Jx;
    double *Dx;
    double delta, gamma;
    /* H_gamma lower, CSC, original order */
    i64 *Ap; i32 *Ai; double *Ax;
    /* factor of P H_gamma P^T = L L^T, L in CSC, permuted order */
    i32 *perm, *iperm;     /* perm[k] = original index of pivot k */
    i64 *Lp; i32 *Li; double *Lx;
    int factored;
} orc;

static void *xmalloc(size_t s) { void *p = malloc(s ? s : 1); if (!p) abort(); return p; }
static void *xcalloc(size_t n, size_t s) { void *p = calloc(n ? n : 1, s ? s : 1); if (!p) abort(); return p; }

typedef struct { i64 row, col; double v; i64 seq; } trip;

static int trip_cmp(const void *a, const void *b) {
    const trip *x = a, *y = b;
    if (x->col != y->col) return x->col < y->col ? -1 : 1;
    if (x->row != y->row) return x->row < y->row ? -1 : 1;
    return x->seq < y->seq ? -1 : (x->seq > y->seq);
}

/* H_gamma = tril(H) + diag(D_x + delta) + gamma * tril(J^T J), Sec. 3 and
 * eq. eq:gamma, as a lower CSC with duplicates summed in a fixed order. */
static void assemble(orc *s) {
    i64 n = s->n, m = s->m;
    i64 cnt = s->Hp[n] + n;
    for (i64 i = 0; i < m; i++) { i64 k = s->Jp[i + 1] - s->Jp[i]; cnt += k * (k + 1) / 2; }
    trip *t = xmalloc(sizeof(trip) * (size_t)cnt);
    i64 q = 0;
    for (i64 i = 0; i < n; i++)
        for (i64 p = s->Hp[i]; p < s->Hp[i + 1]; p++) {
            t[q].row = i; t[q].col = s->Hi[p]; t[q].v = s->Hx[p]; t[q].seq = q; q++;
        }
    for (i64 j = 0; j < n; j++) { t[q].row = j; t[q].col = j; t[q].v = s->Dx[j] + s->delta; t[q].seq = q; q++; }
    for (i64 i = 0; i < m; i++)
        for (i64 a = s->Jp[i]; a < s->Jp[i + 1]; a++)
            for (i64 b = s->Jp[i]; b < s->Jp[i + 1]; b++) {
                i64 pa = s->Ji[a], pb = s->Ji[b];
                if (pa < pb) continue;       /* lower triangle: row >= col */
                t[q].row = pa; t[q].col = pb; t[q].v = s->gamma * s->Jx[a] * s->Jx[b]; t[q].seq = q; q++;
            }
    qsort(t, (size_t)q, sizeof(trip), trip_cmp);
    s->Ap = xcalloc((size_t)n + 1, sizeof(i64));
    s->Ai = xmalloc(sizeof(i32) * (size_t)q);
    s->Ax = xmalloc(sizeof(double) * (size_t)q);
    i64 nz = 0;
    for (i64 k = 0; k < q; k++) {
        if (nz > 0 && s->Ai[nz - 1] == t[k].row && (k > 0 && t[k - 1].col == t[k].col)) {
            s->Ax[nz - 1] += t[k].v;
        } else {
            s->Ai[nz] = (i32)t[k].row; s->Ax[nz] = t[k].v; s->Ap[t[k].col + 1]++; nz++;
        }
    }
    for (i64 j = 0; j < n; j++) s->Ap[j + 1] += s->Ap[j];
    free(t);
}

orc *orc_new(i64 n, i64 m, const i64 *Hp, const i32 *Hi, const double *Hx, const double *Dx,
             const i64 *Jp, const i32 *Ji, const double *Jx, double delta, double gamma) {
    orc *s = xcalloc(1, sizeof(orc));
    s->n = n; s->m = m; s->delta = delta; s->gamma = gamma;
    s->Hp = xmalloc(sizeof(i64) * (size_t)(n + 1)); memcpy(s->Hp, Hp, sizeof(i64) * (size_t)(n + 1));
    s->Hi = xmalloc(sizeof(i32) * (size_t)Hp[n]); memcpy(s->Hi, Hi, sizeof(i32) * (size_t)Hp[n]);
    s->Hx = xmalloc(sizeof(double) * (size_t)Hp[n]); memcpy(s->Hx, Hx, sizeof(double) * (size_t)Hp[n]);
    s->Jp = xmalloc(sizeof(i64) * (size_t)(m + 1)); memcpy(s->Jp, Jp, sizeof(i64) * (size_t)(m + 1));
    s->Ji = xmalloc(sizeof(i32) * (size_t)Jp[m]); memcpy(s->Ji, Ji, sizeof(i32) * (size_t)Jp[m]);
    s->Jx = xmalloc(sizeof(double) * (size_t)Jp[m]); memcpy(s->Jx, Jx, sizeof(double) * (size_t)Jp[m]);
    s->Dx = xmalloc(sizeof(double) * (size_t)n); memcpy(s->Dx, Dx, sizeof(double) * (size_t)n);
    assemble(s);
    return s;
}

static void free_factor(orc *s) {
    free(s->perm); free(s->iperm); free(s->Lp); free(s->Li); free(s->Lx);
    s->perm = s->iperm = NULL; s->Lp = NULL; s->Li = NULL; s->Lx = NULL; s->factored = 0;
}

void orc_free(orc *s) {
    if (!s) return;
    free_factor(s);
    free(s->Hp); free(s->Hi); free(s->Hx); free(s->Jp); free(s->Ji); free(s->Jx); free(s->Dx);
    free(s->Ap); free(s->Ai); free(s->Ax);
    free(s);
}

i64 orc_hgamma_nnz(const orc *s) { return s->Ap[s->n]; }

void orc_hgamma(const orc *s, i64 *colptr, i32 *rowind, double *val) {
    memcpy(colptr, s->Ap, sizeof(i64) * (size_t)(s->n + 1));
    memcpy(rowind, s->Ai, sizeof(i32) * (size_t)s->Ap[s->n]);
    memcpy(val, s->Ax, sizeof(double) * (size_t)s->Ap[s->n]);
}

/* ------------------------------------------------------------------ */
/* exact minimum degree on the explicit elimination graph               */
/* (any fill-reducing order gives the same solution in exact arithmetic;  */
/*  the paper uses AMD, Sec. 5.3; this is the plain exact variant)        */
/* ------------------------------------------------------------------ */

typedef struct { i32 *v; i32 len, cap; } ivec;
static void iv_push(ivec *a, i32 x) {
    if (a->len == a->cap) { a->cap = a->cap ? a->cap * 2 : 4; a->v = realloc(a->v, sizeof(i32) * (size_t)a->cap); if (!a->v) abort(); }
    a->v[a->len++] = x;
}

typedef struct { i64 key; i32 node; } hent;
typedef struct { hent *h; i64 len, cap; } heap;
static void hp_push(heap *H, i64 key, i32 node) {
    if (H->len == H->cap) { H->cap = H->cap ? H->cap * 2 : 64; H->h = realloc(H->h, sizeof(hent) * (size_t)H->cap); if (!H->h) abort(); }
    i64 i = H->len++;
    H->h[i].key = key; H->h[i].node = node;
    while (i > 0) {
        i64 p = (i - 1) / 2;
        if (H->h[p].key < H->h[i].key || (H->h[p].key == H->h[i].key && H->h[p].node <= H->h[i].node)) break;
        hent tmp = H->h[p]; H->h[p] = H->h[i]; H->h[i] = tmp; i = p;
    }
}
static hent hp_pop(heap *H) {
    hent top = H->h[0];
    H->h[0] = H->h[--H->len];
    i64 i = 0;
    for (;;) {
        i64 l = 2 * i + 1, r = l + 1, b = i;
        if (l < H->len && (H->h[l].key < H->h[b].key || (H->h[l].key == H->h[b].key && H->h[l].node < H->h[b].node))) b = l;
        if (r < H->len && (H->h[r].key < H->h[b].key || (H->h[r].key == H->h[b].key && H->h[r].node < H->h[b].node))) b = r;
        if (b == i) break;
        hent tmp = H->h[b]; H->h[b] = H->h[i]; H->h[i] = tmp; i = b;
    }
    return top;
}

/* perm[k] = original index of the k-th eliminated node; ties -> smallest index */
void orc_order_mindeg(const orc *s, i32 *perm) {
    i64 n = s->n;
    ivec *adj = xcalloc((size_t)n, sizeof(ivec));
    for (i64 j = 0; j < n; j++)
        for (i64 p = s->Ap[j]; p < s->Ap[j + 1]; p++) {
            i32 i = s->Ai[p];
            if (i == j) continue;
            iv_push(&adj[i], (i32)j); iv_push(&adj[j], i);
        }
    char *gone = xcalloc((size_t)n, 1);
    i64 *mark = xmalloc(sizeof(i64) * (size_t)n);
    for (i64 i = 0; i < n; i++) mark[i] = -1;
    /* dedupe initial lists */
    for (i64 i = 0; i < n; i++) {
        i32 w = 0;
        for (i32 k = 0; k < adj[i].len; k++) { i32 u = adj[i].v[k]; if (mark[u] != i) { mark[u] = i; adj[i].v[w++] = u; } }
        adj[i].len = w;
    }
    for (i64 i = 0; i < n; i++) mark[i] = -1;
    heap H = {0};
    for (i64 i = 0; i < n; i++) hp_push(&H, adj[i].len, (i32)i);
    i32 *nbr = xmalloc(sizeof(i32) * (size_t)(n ? n : 1));
    i64 stamp = 0;
    for (i64 k = 0; k < n; k++) {
        i32 v;
        for (;;) {
            hent e = hp_pop(&H);
            if (!gone[e.node] && e.key == adj[e.node].len) { v = e.node; break; }
        }
        perm[k] = v; gone[v] = 1;
        /* live neighbours of v */
        i32 nn = 0;
        for (i32 q = 0; q < adj[v].len; q++) { i32 u = adj[v].v[q]; if (!gone[u]) nbr[nn++] = u; }
        free(adj[v].v); adj[v].v = NULL; adj[v].len = adj[v].cap = 0;
        /* make the neighbours a clique; drop v from their lists */
        for (i32 a = 0; a < nn; a++) {
            i32 u = nbr[a];
            stamp++;
            i32 w = 0;
            for (i32 q = 0; q < adj[u].len; q++) {
                i32 t = adj[u].v[q];
                if (t == v || gone[t]) continue;
                if (mark[t] == stamp) continue;
                mark[t] = stamp; adj[u].v[w++] = t;
            }
            adj[u].len = w;
            mark[u] = stamp;
            for (i32 b = 0; b < nn; b++) { i32 t = nbr[b]; if (mark[t] != stamp) { mark[t] = stamp; iv_push(&adj[u], t); } }
            hp_push(&H, adj[u].len, u);
        }
    }
    free(nbr); free(H.h); free(mark); free(gone);
    for (i64 i = 0; i < n; i++) free(adj[i].v);
    free(adj);
}

/* ------------------------------------------------------------------ */
/* left-looking column Cholesky  P H_gamma P^T = L L^T                  */
/* (Cholesky is stable without pivoting, Sec. 3; a non-positive or       */
/*  non-finite pivot means H_gamma is not SPD, the failed-factorization  */
/*  branch of Algorithm 1)                                               */
/* ------------------------------------------------------------------ */

static int cmp_i32(const void *a, const void *b) { i32 x = *(const i32 *)a, y = *(const i32 *)b; return (x > y) - (x < y); }

/* returns 0 on success, 1 if not SPD; *fail_col = original index of the first
 * failing pivot in elimination order (or -1) */
int orc_factor(orc *s, const i32 *perm_in, i64 *fail_col) {
    i64 n = s->n;
    free_factor(s);
    s->perm = xmalloc(sizeof(i32) * (size_t)(n ? n : 1));
    s->iperm = xmalloc(sizeof(i32) * (size_t)(n ? n : 1));
    for (i64 k = 0; k < n; k++) s->perm[k] = perm_in ? perm_in[k] : (i32)k;
    for (i64 k = 0; k < n; k++) s->iperm[s->perm[k]] = (i32)k;
    /* C = P A P^T, lower CSC */
    i64 nzA = s->Ap[n];
    i64 *Cp = xcalloc((size_t)n + 1, sizeof(i64));
    for (i64 j = 0; j < n; j++)
        for (i64 p = s->Ap[j]; p < s->Ap[j + 1]; p++) {
            i64 a = s->iperm[s->Ai[p]], b = s->iperm[j];
            Cp[(a < b ? a : b) + 1]++;
        }
    for (i64 j = 0; j < n; j++) Cp[j + 1] += Cp[j];
    i64 *fill = xmalloc(sizeof(i64) * (size_t)(n ? n : 1));
    for (i64 j = 0; j < n; j++) fill[j] = Cp[j];
    i32 *Ci = xmalloc(sizeof(i32) * (size_t)(nzA ? nzA : 1));
    double *Cx = xmalloc(sizeof(double) * (size_t)(nzA ? nzA : 1));
    for (i64 j = 0; j < n; j++)
        for (i64 p = s->Ap[j]; p < s->Ap[j + 1]; p++) {
            i64 a = s->iperm[s->Ai[p]], b = s->iperm[j];
            i64 lo = a < b ? a : b, hi = a < b ? b : a;
            Ci[fill[lo]] = (i32)hi; Cx[fill[lo]] = s->Ax[p]; fill[lo]++;
        }
    free(fill);

    i64 cap = nzA + n + 16, nz = 0;
    s->Lp = xcalloc((size_t)n + 1, sizeof(i64));
    s->Li = xmalloc(sizeof(i32) * (size_t)cap);
    s->Lx = xmalloc(sizeof(double) * (size_t)cap);
    double *w = xcalloc((size_t)(n ? n : 1), sizeof(double));
    char *mk = xcalloc((size_t)(n ? n : 1), 1);
    i32 *pat = xmalloc(sizeof(i32) * (size_t)(n ? n : 1));
    i64 *head = xmalloc(sizeof(i64) * (size_t)(n ? n : 1));   /* linked list of columns k with L(j,k) != 0 */
    i64 *next = xmalloc(sizeof(i64) * (size_t)(n ? n : 1));
    i64 *first = xmalloc(sizeof(i64) * (size_t)(n ? n : 1));  /* next unused position in column k */
    for (i64 j = 0; j < n; j++) head[j] = -1;
    int status = 0;
    *fail_col = -1;
    for (i64 j = 0; j < n; j++) {
        i32 np = 0;
        for (i64 p = Cp[j]; p < Cp[j + 1]; p++) {
            i32 i = Ci[p];
            if (!mk[i]) { mk[i] = 1; pat[np++] = i; w[i] = 0.0; }
            w[i] += Cx[p];
        }
        if (!mk[j]) { mk[j] = 1; pat[np++] = (i32)j; w[j] = 0.0; }
        /* left-looking updates from every column k < j with L(j,k) != 0 */
        i64 k = head[j];
        while (k >= 0) {
            i64 nk = next[k];
            i64 pos = first[k];
            double ljk = s->Lx[pos];
            for (i64 p = pos; p < s->Lp[k + 1]; p++) {
                i32 i = s->Li[p];
                if (!mk[i]) { mk[i] = 1; pat[np++] = i; w[i] = 0.0; }
                w[i] -= s->Lx[p] * ljk;
            }
            first[k] = pos + 1;
            if (first[k] < s->Lp[k + 1]) {
                i32 r = s->Li[first[k]];
                next[k] = head[r]; head[r] = k;
            }
            k = nk;
        }
        double d = w[j];
        if (!(d > 0.0) || !isfinite(d)) {
            status = 1; *fail_col = s->perm[j];
            for (i32 q = 0; q < np; q++) mk[pat[q]] = 0;
            break;
        }
        double ljj = sqrt(d);
        qsort(pat, (size_t)np, sizeof(i32), cmp_i32);   /* pat[0] == j */
        if (nz + np > cap) {
            while (nz + np > cap) cap *= 2;
            s->Li = realloc(s->Li, sizeof(i32) * (size_t)cap); s->Lx = realloc(s->Lx, sizeof(double) * (size_t)cap);
            if (!s->Li || !s->Lx) abort();
        }
        s->Li[nz] = (i32)j; s->Lx[nz] = ljj; nz++;
        for (i32 q = 1; q < np; q++) { s->Li[nz] = pat[q]; s->Lx[nz] = w[pat[q]] / ljj; nz++; }
        for (i32 q = 0; q < np; q++) mk[pat[q]] = 0;
        s->Lp[j + 1] = nz;
        first[j] = s->Lp[j] + 1;
        if (first[j] < s->Lp[j + 1]) { i32 r = s->Li[first[j]]; next[j] = head[r]; head[r] = j; }
    }
    free(w); free(mk); free(pat); free(head); free(next); free(first); free(Cp); free(Ci); free(Cx);
    s->factored = (status == 0);
    return status;
}

i64 orc_L_nnz(const orc *s) { return s->factored ? s->Lp[s->n] : -1; }

void orc_L(const orc *s, i64 *colptr, i32 *rowind, double *val) {
    memcpy(colptr, s->Lp, sizeof(i64) * (size_t)(s->n + 1));
    memcpy(rowind, s->Li, sizeof(i32) * (size_t)s->Lp[s->n]);
    memcpy(val, s->Lx, sizeof(double) * (size_t)s->Lp[s->n]);
}

/* x = H_gamma^{-1} b (original order): forward column-oriented, backward dot form */
void orc_hsolve(const orc *s, const double *b, double *x) {
    i64 n = s->n;
    double *t = xmalloc(sizeof(double) * (size_t)(n ? n : 1));
    for (i64 k = 0; k < n; k++) t[k] = b[s->perm[k]];
    for (i64 j = 0; j < n; j++) {                /* L t = P b */
        t[j] /= s->Lx[s->Lp[j]];
        for (i64 p = s->Lp[j] + 1; p < s->Lp[j + 1]; p++) t[s->Li[p]] -= s->Lx[p] * t[j];
    }
    for (i64 j = n - 1; j >= 0; j--) {           /* L^T u = t */
        double a = t[j];
        for (i64 p = s->Lp[j] + 1; p < s->Lp[j + 1]; p++) a -= s->Lx[p] * t[s->Li[p]];
        t[j] = a / s->Lx[s->Lp[j]];
    }
    for (i64 k = 0; k < n; k++) x[s->perm[k]] = t[k];
    free(t);
}

/* ------------------------------------------------------------------ */
/* operators                                                           */
/* ------------------------------------------------------------------ */

static void J_mul(const orc *s, const double *v, double *out) {          /* out = J v */
    for (i64 i = 0; i < s->m; i++) {
        double a = 0.0;
        for (i64 p = s->Jp[i]; p < s->Jp[i + 1]; p++) a += s->Jx[p] * v[s->Ji[p]];
        out[i] = a;
    }
}
static void JT_mul(const orc *s, const double *v, double *out) {         /* out = J^T v */
    for (i64 j = 0; j < s->n; j++) out[j] = 0.0;
    for (i64 i = 0; i < s->m; i++)
        for (i64 p = s->Jp[i]; p < s->Jp[i + 1]; p++) out[s->Ji[p]] += s->Jx[p] * v[i];
}
static void H_mul(const orc *s, const double *v, double *out) {          /* out = H v, from tril(H) */
    for (i64 j = 0; j < s->n; j++) out[j] = 0.0;
    for (i64 i = 0; i < s->n; i++)
        for (i64 p = s->Hp[i]; p < s->Hp[i + 1]; p++) {
            i64 j = s->Hi[p];
            out[i] += s->Hx[p] * v[j];
            if (j != i) out[j] += s->Hx[p] * v[i];
        }
}
static double dot(const double *a, const double *b, i64 n) { double s = 0.0; for (i64 i = 0; i < n; i++) s += a[i] * b[i]; return s; }
static double nrm2(const double *a, i64 n) { return sqrt(dot(a, a, n)); }

/* ------------------------------------------------------------------ */
/* compensated residual (Ogita, Rump, Oishi 2005: TwoSum, TwoProduct by  */
/* FMA, Dot2). Each row keeps an unevaluated sum hi + lo; a term a*b is  */
/* split exactly into fl(a*b) + err and both parts are accumulated, so   */
/* the rounded row sum is within about u of the exact one.               */
/* ------------------------------------------------------------------ */

/* a + b = *s + *e exactly (Knuth's TwoSum, no ordering assumption) */
static void two_sum(double a, double b, double *s, double *e) {
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

/* a * b = *p + *e exactly (FMA form of TwoProduct) */
static void two_prod(double a, double b, double *p, double *e) {
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

typedef struct { double hi, lo; } acc2;

/* acc += a * b (Dot2 step: the product's error and the sum's error both go
 * to the low part) */
static void acc_fma(acc2 *c, double a, double b) {
    double p, ep, s, es;
    two_prod(a, b, &p, &ep);
    two_sum(c->hi, p, &s, &es);
    c->hi = s;
    c->lo += es + ep;
}

static void acc_add(acc2 *c, double a) {
    double s, es;
    two_sum(c->hi, a, &s, &es);
    c->hi = s;
    c->lo += es;
}

/* res = r - K (z + z_lo), K = [H + D_x + delta I, J^T; J, 0], row by row with
 * compensated sums (z_lo = the low parts of a double-double iterate, or
 * NULL); t (if non-NULL) gets per row |r_i| + the sum of |term| over the
 * row's terms (|K||z| + |r| when diag(H) >= 0, which makes every diagonal
 * term of K of one sign). */
static void residual_comp(const orc *s, const double *r1, const double *r2, const double *x, const double *y,
                          const double *xl, const double *yl, double *res1, double *res2, double *t1, double *t2) {
    i64 n = s->n, m = s->m;
    acc2 *a1 = xcalloc((size_t)(n ? n : 1), sizeof(acc2)), *a2 = xcalloc((size_t)(m ? m : 1), sizeof(acc2));
    double *f1 = xcalloc((size_t)(n ? n : 1), sizeof(double)), *f2 = xcalloc((size_t)(m ? m : 1), sizeof(double));
    for (i64 i = 0; i < n; i++) { a1[i].hi = r1[i]; f1[i] = fabs(r1[i]); }
    for (i64 i = 0; i < m; i++) { a2[i].hi = r2[i]; f2[i] = fabs(r2[i]); }
    /* H (tril stored; the upper entries are the transposes) */
    for (i64 i = 0; i < n; i++)
        for (i64 p = s->Hp[i]; p < s->Hp[i + 1]; p++) {
            i64 j = s->Hi[p];
            double h = s->Hx[p];
            acc_fma(&a1[i], -h, x[j]); f1[i] += fabs(h * x[j]);
            if (xl) acc_fma(&a1[i], -h, xl[j]);
            if (j != i) {
                acc_fma(&a1[j], -h, x[i]); f1[j] += fabs(h * x[i]);
                if (xl) acc_fma(&a1[j], -h, xl[i]);
            }
        }
    /* D_x and delta on the diagonal, each a term of its own */
    for (i64 i = 0; i < n; i++) {
        acc_fma(&a1[i], -s->Dx[i], x[i]); f1[i] += fabs(s->Dx[i] * x[i]);
        acc_fma(&a1[i], -s->delta, x[i]); f1[i] += fabs(s->delta * x[i]);
        if (xl) { acc_fma(&a1[i], -s->Dx[i], xl[i]); acc_fma(&a1[i], -s->delta, xl[i]); }
    }
    /* J^T y into the first block, J x into the second */
    for (i64 k = 0; k < m; k++)
        for (i64 p = s->Jp[k]; p < s->Jp[k + 1]; p++) {
            i64 j = s->Ji[p];
            double v = s->Jx[p];
            acc_fma(&a1[j], -v, y[k]); f1[j] += fabs(v * y[k]);
            acc_fma(&a2[k], -v, x[j]); f2[k] += fabs(v * x[j]);
            if (yl) acc_fma(&a1[j], -v, yl[k]);
            if (xl) acc_fma(&a2[k], -v, xl[j]);
        }
    for (i64 i = 0; i < n; i++) res1[i] = a1[i].hi + a1[i].lo;
    for (i64 i = 0; i < m; i++) res2[i] = a2[i].hi + a2[i].lo;
    if (t1) memcpy(t1, f1, sizeof(double) * (size_t)n);
    if (t2) memcpy(t2, f2, sizeof(double) * (size_t)m);
    free(a1); free(a2); free(f1); free(f2);
}

/* res = r - K z (compensated) */
static void kkt_residual(const orc *s, const double *r1, const double *r2, const double *x, const double *y,
                         double *res1, double *res2) {
    residual_comp(s, r1, r2, x, y, NULL, NULL, res1, res2, NULL, NULL);
}

/* exposed for the pins: the compensated residual and the per-row term sums */
void orc_residual(const orc *s, const double *r1, const double *r2, const double *x, const double *y,
                  double *res1, double *res2, double *t1, double *t2) {
    residual_comp(s, r1, r2, x, y, NULL, NULL, res1, res2, t1, t2);
}

/* ||K||_inf: max row sum of |K| */
static double kkt_norm_inf(const orc *s) {
    i64 n = s->n, m = s->m;
    double *rs = xcalloc((size_t)(n + m ? n + m : 1), sizeof(double));
    for (i64 i = 0; i < n; i++)
        for (i64 p = s->Hp[i]; p < s->Hp[i + 1]; p++) {
            i64 j = s->Hi[p];
            if (j == i) rs[i] += fabs(s->Hx[p] + s->Dx[i] + s->delta);
            else { rs[i] += fabs(s->Hx[p]); rs[j] += fabs(s->Hx[p]); }
        }
    for (i64 i = 0; i < n; i++) {  /* diagonals absent from the tril(H) pattern */
        int has = 0;
        for (i64 p = s->Hp[i]; p < s->Hp[i + 1]; p++) if (s->Hi[p] == i) has = 1;
        if (!has) rs[i] += fabs(s->Dx[i] + s->delta);
    }
    for (i64 i = 0; i < m; i++)
        for (i64 p = s->Jp[i]; p < s->Jp[i + 1]; p++) { rs[n + i] += fabs(s->Jx[p]); rs[s->Ji[p]] += fabs(s->Jx[p]); }
    double mx = 0.0;
    for (i64 i = 0; i < n + m; i++) if (rs[i] > mx) mx = rs[i];
    free(rs);
    return mx;
}

/* RR, BE (Sec. 5.1, ||K||_inf for ||K||_2) of the compensated residual, and
 * the plain FP64 evaluation floor u * || |K||z| + |r| ||_2 / ||r||_2
 * (u = 2^-53; |K||z| summed term by term as above). */
void orc_metrics(orc *s, const double *r1, const double *r2, const double *x, const double *y, double *out3) {
    i64 n = s->n, m = s->m;
    double *a = xmalloc(sizeof(double) * (size_t)(n ? n : 1)), *b = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    double *f1 = xmalloc(sizeof(double) * (size_t)(n ? n : 1)), *f2 = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    residual_comp(s, r1, r2, x, y, NULL, NULL, a, b, f1, f2);
    double rn = sqrt(dot(a, a, n) + dot(b, b, m));
    double bn = sqrt(dot(r1, r1, n) + dot(r2, r2, m));
    double zn = sqrt(dot(x, x, n) + dot(y, y, m));
    double kn = kkt_norm_inf(s);
    double fl = ldexp(1.0, -53) * sqrt(dot(f1, f1, n) + dot(f2, f2, m));
    out3[0] = bn > 0 ? rn / bn : rn;
    out3[1] = rn / (kn * zn + bn);
    out3[2] = bn > 0 ? fl / bn : fl;
    free(a); free(b); free(f1); free(f2);
}

/* ------------------------------------------------------------------ */
/* hybrid solve: Algorithm 1 solve phase + FP64 refinement             */
/* ------------------------------------------------------------------ */

typedef struct {
    double cg_tol;        /* 1e-12 */
    double kkt_tol;       /* 1e-10 */
    double qf_eps;        /* 1e-14 */
    double delta2;        /* used only after a breakdown; 0 = report breakdown */
    i64 max_cg;           /* <= 0: min(m, 1000) */
    i64 max_refine;       /* 10 */
    i64 inexact;          /* 1: passes after the first at the CG tolerance pass_tol() gives */
} orc_opts;

/* Inexact refinement (a reading: the paper has no refinement): a pass after
 * the first needs its correction only as accurately as it takes RR below
 * kkt_tol with a tenfold margin, so its CG stops at the relative residual
 * max(cg_tol, min(1e-2, 0.1 * kkt_tol / RR)) with RR that of the current
 * iterate. */
static orc_opts pass_opts(const orc_opts *o, i64 pass, double rr) {
    orc_opts q = *o;
    if (o->inexact && pass > 0 && rr > 0.0) {
        double t = 0.1 * o->kkt_tol / rr;
        if (t > 1e-2) t = 1e-2;
        if (t > q.cg_tol) q.cg_tol = t;
    }
    return q;
}

typedef struct {
    i64 status;           /* 0 ok, 2 CG breakdown, 3 not converged, -3 no factor */
    i64 passes;           /* hybrid passes run (1 + refinement steps) */
    i64 cg_iters[16];     /* CG iterations per pass */
    double rr_hist[16];   /* RR after each pass */
    double rr, be, floor;
    i64 inertia[3];
} orc_report;

/* one hybrid pass: (x, y) ~= K^{-1} (r1, r2); returns CG iterations, or -1 on
 * breakdown with delta2 == 0 */
static i64 hybrid_pass(const orc *s, const orc_opts *o, const double *r1, const double *r2, double *x, double *y,
                       int *breakdown) {
    i64 n = s->n, m = s->m;
    double *rhat = xmalloc(sizeof(double) * (size_t)(n ? n : 1));
    double *w = xmalloc(sizeof(double) * (size_t)(n ? n : 1));
    double *t = xmalloc(sizeof(double) * (size_t)(n ? n : 1));
    double *u = xmalloc(sizeof(double) * (size_t)(n ? n : 1));
    double *bv = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    double *res = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    double *p = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    double *q = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    *breakdown = 0;
    /* rhat = r1 + gamma J^T r2 */
    JT_mul(s, r2, t);
    for (i64 j = 0; j < n; j++) rhat[j] = r1[j] + s->gamma * t[j];
    /* w = H_gamma^{-1} rhat ;  b = J w - r2 */
    orc_hsolve(s, rhat, w);
    J_mul(s, w, bv);
    for (i64 i = 0; i < m; i++) bv[i] -= r2[i];
    /* CG on S y = b, y0 = 0 */
    i64 max_cg = o->max_cg > 0 ? o->max_cg : (m < 1000 ? m : 1000);
    if (max_cg < 1) max_cg = 1;
    for (i64 i = 0; i < m; i++) { y[i] = 0.0; res[i] = bv[i]; p[i] = bv[i]; }
    double bnorm = nrm2(bv, m);
    double rho = dot(res, res, m);
    double curv0 = -1.0;
    i64 it = 0;
    double d2 = 0.0;
    if (m > 0 && bnorm > 0.0) {
        while (it < max_cg) {
            JT_mul(s, p, t);
            orc_hsolve(s, t, u);
            J_mul(s, u, q);
            for (i64 i = 0; i < m; i++) q[i] += d2 * p[i];
            double pq = dot(p, q, m), pp = dot(p, p, m);
            if (curv0 < 0.0) curv0 = pq / pp;
            if (!(pq > o->qf_eps * pp * curv0)) {
                /* quadratic form below the threshold (Algorithm 1's breakdown
                 * test): restart on S + delta2 I */
                *breakdown = 1;
                if (o->delta2 > 0.0 && d2 == 0.0) {
                    d2 = o->delta2;
                    for (i64 i = 0; i < m; i++) { y[i] = 0.0; res[i] = bv[i]; p[i] = bv[i]; }
                    rho = dot(res, res, m); curv0 = -1.0;
                    continue;
                }
                break;
            }
            double alpha = rho / pq;
            for (i64 i = 0; i < m; i++) { y[i] += alpha * p[i]; res[i] -= alpha * q[i]; }
            double rho1 = dot(res, res, m);
            it++;
            if (sqrt(rho1) <= o->cg_tol * bnorm) break;
            double beta = rho1 / rho;
            rho = rho1;
            for (i64 i = 0; i < m; i++) p[i] = res[i] + beta * p[i];
        }
    }
    /* x = H_gamma^{-1} (rhat - J^T y) */
    JT_mul(s, y, t);
    for (i64 j = 0; j < n; j++) t[j] = rhat[j] - t[j];
    orc_hsolve(s, t, x);
    free(rhat); free(w); free(t); free(u); free(bv); free(res); free(p); free(q);
    return it;
}

int orc_solve(orc *s, const orc_opts *o, const double *r1, const double *r2, double *x, double *y, orc_report *rep) {
    i64 n = s->n, m = s->m;
    memset(rep, 0, sizeof(*rep));
    if (!s->factored) { rep->status = -3; return -3; }
    double *ex = xmalloc(sizeof(double) * (size_t)(n ? n : 1)), *ey = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    double *g1 = xmalloc(sizeof(double) * (size_t)(n ? n : 1)), *g2 = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    double rn = sqrt(dot(r1, r1, n) + dot(r2, r2, m));
    for (i64 j = 0; j < n; j++) { x[j] = 0.0; g1[j] = r1[j]; }
    for (i64 i = 0; i < m; i++) { y[i] = 0.0; g2[i] = r2[i]; }
    i64 max_ref = o->max_refine > 0 ? o->max_refine : 10;
    if (max_ref > 15) max_ref = 15;
    int brk_any = 0;
    double rr = rn > 0 ? 1.0 : 0.0, rr_best = INFINITY;
    i64 pass = 0;
    while (pass <= max_ref) {
        int brk = 0;
        const orc_opts po = pass_opts(o, pass, rr);
        i64 it = hybrid_pass(s, &po, g1, g2, ex, ey, &brk);
        brk_any |= brk;
        for (i64 j = 0; j < n; j++) x[j] += ex[j];
        for (i64 i = 0; i < m; i++) y[i] += ey[i];
        kkt_residual(s, r1, r2, x, y, g1, g2);
        rr = rn > 0 ? sqrt(dot(g1, g1, n) + dot(g2, g2, m)) / rn : 0.0;
        rep->cg_iters[pass] = it;
        rep->rr_hist[pass] = rr;
        pass++;
        if (rr <= o->kkt_tol || brk) break;
        /* a later pass that does not halve RR: z is as close to the exact
         * solution as FP64 entries allow (the residual of the rounded
         * solution is of the order of the floor) */
        if (pass >= 2 && !(rr < 0.5 * rr_best)) break;
        if (rr < rr_best) rr_best = rr;
    }
    rep->passes = pass;
    double mt[3];
    orc_metrics(s, r1, r2, x, y, mt);
    rep->rr = mt[0]; rep->be = mt[1]; rep->floor = mt[2];
    /* Theorem 3 with congruence + Haynsworth: n_x positive eigenvalues from the
     * Cholesky of H_gamma; the rest are those of -S, negative unless J is
     * rank-deficient. A breakdown shows S singular (or nearly so) but not its
     * nullity, so negative and zero counts are then left undetermined (-1). */
    rep->inertia[0] = n; rep->inertia[1] = brk_any ? -1 : m; rep->inertia[2] = brk_any ? -1 : 0;
    rep->status = brk_any && o->delta2 == 0.0 ? 2 : (rr <= o->kkt_tol ? 0 : 3);
    free(ex); free(ey); free(g1); free(g2);
    return (int)rep->status;
}

/* Refinement with the iterate held as an unevaluated sum z + z_lo of two
 * doubles (z_lo starts at 0): each step evaluates g = r - K (z + z_lo) with
 * compensated sums, takes the correction e from one hybrid pass on g, and
 * adds it with TwoSum per entry, renormalised so that z = fl(z + z_lo). The
 * steps stop after max_steps or when ||g|| no longer halves. On return
 * (x, y) = z, the exact solution rounded to FP64 up to the accuracy the
 * steps reached; hist[k] = ||g|| / ||r|| before step k (max_steps + 1
 * entries). Returns the number of steps taken. */
i64 orc_refine_dd(orc *s, const orc_opts *o, const double *r1, const double *r2, double *x, double *y,
                  i64 max_steps, double *hist) {
    i64 n = s->n, m = s->m;
    if (!s->factored) return -3;
    double *xl = xcalloc((size_t)(n ? n : 1), sizeof(double)), *yl = xcalloc((size_t)(m ? m : 1), sizeof(double));
    double *ex = xmalloc(sizeof(double) * (size_t)(n ? n : 1)), *ey = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    double *g1 = xmalloc(sizeof(double) * (size_t)(n ? n : 1)), *g2 = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    double rn = sqrt(dot(r1, r1, n) + dot(r2, r2, m));
    if (!(rn > 0)) rn = 1.0;
    double prev = INFINITY;
    i64 k = 0;
    for (;; k++) {
        residual_comp(s, r1, r2, x, y, xl, yl, g1, g2, NULL, NULL);
        double g = sqrt(dot(g1, g1, n) + dot(g2, g2, m)) / rn;
        if (hist) hist[k] = g;
        if (k >= max_steps || !(g < 0.5 * prev) || g == 0.0) break;
        prev = g;
        int brk = 0;
        hybrid_pass(s, o, g1, g2, ex, ey, &brk);
        for (i64 j = 0; j < n + m; j++) {
            double *hi = j < n ? &x[j] : &y[j - n], *lo = j < n ? &xl[j] : &yl[j - n];
            double e = j < n ? ex[j] : ey[j - n];
            double sh, sl;
            two_sum(*hi, e, &sh, &sl);
            sl += *lo;
            two_sum(sh, sl, hi, lo);   /* renormalise: hi = fl(sh + sl) */
        }
    }
    free(xl); free(yl); free(ex); free(ey); free(g1); free(g2);
    return k;
}

/* single hybrid pass without refinement (for CG-count and Theorem 4 tests) */
i64 orc_hybrid_once(orc *s, const orc_opts *o, const double *r1, const double *r2, double *x, double *y, int *breakdown) {
    if (!s->factored) return -3;
    return hybrid_pass(s, o, r1, r2, x, y, breakdown);
}

/* plain operator applications, exposed so tests can check them against
 * dense matrices */
void orc_apply_K(const orc *s, const double *x, const double *y, double *o1, double *o2) {
    i64 n = s->n, m = s->m;
    double *z1 = xcalloc((size_t)(n ? n : 1), sizeof(double)), *z2 = xcalloc((size_t)(m ? m : 1), sizeof(double));
    kkt_residual(s, z1, z2, x, y, o1, o2);
    for (i64 j = 0; j < n; j++) o1[j] = -o1[j];
    for (i64 i = 0; i < m; i++) o2[i] = -o2[i];
    free(z1); free(z2);
}

/* ------------------------------------------------------------------ */
/* Algorithm 1's regularization of the (1,1) block, and the gamma      */
/* heuristic of Sec. 3                                                 */
/* ------------------------------------------------------------------ */

/* K's (1,1) block regularization becomes delta (re-assembles H_gamma; the
 * factor is dropped). */
void orc_set_delta(orc *s, double delta) {
    free_factor(s);
    free(s->Ap); free(s->Ai); free(s->Ax);
    s->Ap = NULL; s->Ai = NULL; s->Ax = NULL;
    s->delta = delta;
    assemble(s);
}

/* Algorithm 1, Sec. 4.1: Cholesky of H_gamma with the system's delta; while
 * it fails and delta1 <= delta_max / 2, the first retry takes delta1 =
 * delta_min, every later one doubles delta_min and takes delta1 = delta_min
 * (so delta_min carries the last value tried into the next matrix of a
 * sequence). The system keeps delta + delta1 as its (1,1) regularization:
 * the solve then works on the perturbed system, as Algorithm 1's solves
 * do. Returns 0 (factored) or 1 (still not positive definite: the caller's
 * fail-safe), with *delta1 the last value tried and *fail_col the failing
 * pivot of the last attempt. */
int orc_factor_regularized(orc *s, const i32 *perm, double *delta_min, double delta_max, double *delta1,
                           i64 *fail_col) {
    const double base = s->delta;
    double d1 = 0.0;
    int st = orc_factor(s, perm, fail_col);
    while (st != 0 && d1 <= delta_max / 2) {
        if (d1 == 0.0) d1 = *delta_min;
        else { *delta_min = 2.0 * *delta_min; d1 = *delta_min; }
        orc_set_delta(s, base + d1);
        st = orc_factor(s, perm, fail_col);
    }
    *delta1 = d1;
    return st;
}

/* gamma = ||Htilde|| / ||J||^2 (Sec. 3, after Golub and Greif), with the
 * infinity norm standing in for the 2-norm as in Sec. 5.1 and Htilde the
 * system's (1,1) block H + D_x + delta I. Returns 0 when J is empty or
 * zero. */
double orc_gamma_heuristic(const orc *s) {
    i64 n = s->n, m = s->m;
    double *rs = xcalloc((size_t)(n ? n : 1), sizeof(double));
    for (i64 i = 0; i < n; i++) {
        int has = 0;
        for (i64 p = s->Hp[i]; p < s->Hp[i + 1]; p++) {
            i64 j = s->Hi[p];
            if (j == i) { rs[i] += fabs(s->Hx[p] + s->Dx[i] + s->delta); has = 1; }
            else { rs[i] += fabs(s->Hx[p]); rs[j] += fabs(s->Hx[p]); }
        }
        if (!has) rs[i] += fabs(s->Dx[i] + s->delta);
    }
    double hn = 0.0, jn = 0.0;
    for (i64 i = 0; i < n; i++) if (rs[i] > hn) hn = rs[i];
    for (i64 i = 0; i < m; i++) {
        double r = 0.0;
        for (i64 p = s->Jp[i]; p < s->Jp[i + 1]; p++) r += fabs(s->Jx[p]);
        if (r > jn) jn = r;
    }
    free(rs);
    return jn > 0.0 ? hn / (jn * jn) : 0.0;
}

/* ------------------------------------------------------------------ */
/* symmetrized Ruiz scaling (Sec. 4.1, after Ruiz 2001)                */
/* ------------------------------------------------------------------ */

/* d (n + m entries) such that D K D, D = diag(d), has every row's largest
 * magnitude near 1: starting from d = 1, each of `iters` sweeps divides d_i
 * by the square root of row i's largest |(D K D)_ij| (rows that are all
 * zero keep their d). K = [H + D_x + delta I, J^T; J, 0] as in the solve. */
void orc_ruiz(const orc *s, i64 iters, double *d) {
    i64 n = s->n, m = s->m;
    double *r = xmalloc(sizeof(double) * (size_t)(n + m ? n + m : 1));
    for (i64 i = 0; i < n + m; i++) d[i] = 1.0;
    for (i64 it = 0; it < iters; it++) {
        for (i64 i = 0; i < n + m; i++) r[i] = 0.0;
        for (i64 i = 0; i < n; i++) {
            int has = 0;
            for (i64 p = s->Hp[i]; p < s->Hp[i + 1]; p++) {
                i64 j = s->Hi[p];
                if (j == i) {
                    double a = fabs(s->Hx[p] + s->Dx[i] + s->delta) * d[i] * d[i];
                    if (a > r[i]) r[i] = a;
                    has = 1;
                } else {
                    double a = fabs(s->Hx[p]) * d[i] * d[j];
                    if (a > r[i]) r[i] = a;
                    if (a > r[j]) r[j] = a;
                }
            }
            if (!has) { double a = fabs(s->Dx[i] + s->delta) * d[i] * d[i]; if (a > r[i]) r[i] = a; }
        }
        for (i64 k = 0; k < m; k++)
            for (i64 p = s->Jp[k]; p < s->Jp[k + 1]; p++) {
                i64 j = s->Ji[p];
                double a = fabs(s->Jx[p]) * d[n + k] * d[j];
                if (a > r[n + k]) r[n + k] = a;
                if (a > r[j]) r[j] = a;
            }
        for (i64 i = 0; i < n + m; i++) if (r[i] > 0.0) d[i] /= sqrt(r[i]);
    }
    free(r);
}

/* The system D K D for the scaling d: (1,1) block D1 (H + D_x + delta I) D1
 * with delta folded into the diagonal (D_x' = d1^2 (D_x + delta), delta' =
 * 0), J' = D2 J D1, the same gamma. */
orc *orc_new_scaled(const orc *s, const double *d) {
    i64 n = s->n, m = s->m;
    double *Hs = xmalloc(sizeof(double) * (size_t)(s->Hp[n] ? s->Hp[n] : 1));
    double *Js = xmalloc(sizeof(double) * (size_t)(s->Jp[m] ? s->Jp[m] : 1));
    double *Ds = xmalloc(sizeof(double) * (size_t)(n ? n : 1));
    for (i64 i = 0; i < n; i++)
        for (i64 p = s->Hp[i]; p < s->Hp[i + 1]; p++) Hs[p] = s->Hx[p] * d[i] * d[s->Hi[p]];
    for (i64 k = 0; k < m; k++)
        for (i64 p = s->Jp[k]; p < s->Jp[k + 1]; p++) Js[p] = s->Jx[p] * d[n + k] * d[s->Ji[p]];
    for (i64 i = 0; i < n; i++) Ds[i] = d[i] * d[i] * (s->Dx[i] + s->delta);
    orc *t = orc_new(n, m, s->Hp, s->Hi, Hs, Ds, s->Jp, s->Ji, Js, 0.0, s->gamma);
    free(Hs); free(Js); free(Ds);
    return t;
}

/* Solve K z = r with the hybrid passes on the scaled system (Sec. 4.1: scale,
 * then apply the method with gamma relative to the scaled system) and the
 * refinement on the original K: g = r - K z (compensated); one pass on
 * D K D with right-hand side D g gives e_hat; z += D e_hat. Stop rules,
 * report and inertia as orc_solve (D K D is congruent to K). The scaled
 * system is factored with perm (NULL: natural). Returns the status. */
int orc_solve_scaled(orc *s, const orc_opts *o, const double *d, const i32 *perm, const double *r1,
                     const double *r2, double *x, double *y, orc_report *rep) {
    i64 n = s->n, m = s->m;
    memset(rep, 0, sizeof(*rep));
    orc *t = orc_new_scaled(s, d);
    i64 fc;
    if (orc_factor(t, perm, &fc) != 0) { orc_free(t); rep->status = 1; return 1; }
    double *ex = xmalloc(sizeof(double) * (size_t)(n ? n : 1)), *ey = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    double *g1 = xmalloc(sizeof(double) * (size_t)(n ? n : 1)), *g2 = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    double rn = sqrt(dot(r1, r1, n) + dot(r2, r2, m));
    for (i64 j = 0; j < n; j++) { x[j] = 0.0; g1[j] = r1[j] * d[j]; }
    for (i64 i = 0; i < m; i++) { y[i] = 0.0; g2[i] = r2[i] * d[n + i]; }
    i64 max_ref = o->max_refine > 0 ? o->max_refine : 10;
    if (max_ref > 15) max_ref = 15;
    int brk_any = 0;
    double rr = rn > 0 ? 1.0 : 0.0, rr_best = INFINITY;
    i64 pass = 0;
    while (pass <= max_ref) {
        int brk = 0;
        const orc_opts po = pass_opts(o, pass, rr);
        i64 it = hybrid_pass(t, &po, g1, g2, ex, ey, &brk);
        brk_any |= brk;
        for (i64 j = 0; j < n; j++) x[j] += d[j] * ex[j];
        for (i64 i = 0; i < m; i++) y[i] += d[n + i] * ey[i];
        kkt_residual(s, r1, r2, x, y, g1, g2);
        rr = rn > 0 ? sqrt(dot(g1, g1, n) + dot(g2, g2, m)) / rn : 0.0;
        for (i64 j = 0; j < n; j++) g1[j] *= d[j];
        for (i64 i = 0; i < m; i++) g2[i] *= d[n + i];
        rep->cg_iters[pass] = it;
        rep->rr_hist[pass] = rr;
        pass++;
        if (rr <= o->kkt_tol || brk) break;
        if (pass >= 2 && !(rr < 0.5 * rr_best)) break;
        if (rr < rr_best) rr_best = rr;
    }
    rep->passes = pass;
    double mt[3];
    orc_metrics(s, r1, r2, x, y, mt);
    rep->rr = mt[0]; rep->be = mt[1]; rep->floor = mt[2];
    rep->inertia[0] = n; rep->inertia[1] = brk_any ? -1 : m; rep->inertia[2] = brk_any ? -1 : 0;
    rep->status = brk_any && o->delta2 == 0.0 ? 2 : (rr <= o->kkt_tol ? 0 : 3);
    free(ex); free(ey); free(g1); free(g2);
    orc_free(t);
    return (int)rep->status;
}

/* ------------------------------------------------------------------ */
/* the full 4x4 system of Sec. 3 (eq. linsys4x4)                       */
/* ------------------------------------------------------------------ */
/* K4 = [H + D_x + delta I, 0, J^T, J_d^T; 0, D_s, 0, -I; J, 0, 0, 0;
 *       J_d, -I, 0, 0], unknowns (dx, ds, dy, dyd), right-hand side
 * (rx~, rs, ry, ryd). Eliminating ds = J_d dx - ryd and dyd = D_s ds - rs
 * gives the 2x2 system (eq. linsys2x2) with Htilde = H + D_x + J_d^T D_s J_d
 * and r_x = rx~ + J_d^T (D_s ryd + rs), which the hybrid method solves. */
typedef struct {
    orc *two;                 /* the 2x2 system with Htilde's H part H + J_d^T D_s J_d */
    i64 n, m, md;
    i64 *Hp; i32 *Hi; double *Hx;        /* tril(H) as given */
    i64 *Dp; i32 *Di; double *Dv;        /* J_d CSR */
    double *Ds;
} orc4;

orc4 *orc4_new(i64 n, i64 m, i64 md, const i64 *Hp, const i32 *Hi, const double *Hx, const double *Dx,
               const i64 *Jp, const i32 *Ji, const double *Jx, const i64 *Dp, const i32 *Di, const double *Dv,
               const double *Ds, double delta, double gamma) {
    orc4 *q = xcalloc(1, sizeof(orc4));
    q->n = n; q->m = m; q->md = md;
    q->Hp = xmalloc(sizeof(i64) * (size_t)(n + 1)); memcpy(q->Hp, Hp, sizeof(i64) * (size_t)(n + 1));
    q->Hi = xmalloc(sizeof(i32) * (size_t)(Hp[n] ? Hp[n] : 1)); memcpy(q->Hi, Hi, sizeof(i32) * (size_t)Hp[n]);
    q->Hx = xmalloc(sizeof(double) * (size_t)(Hp[n] ? Hp[n] : 1)); memcpy(q->Hx, Hx, sizeof(double) * (size_t)Hp[n]);
    q->Dp = xmalloc(sizeof(i64) * (size_t)(md + 1)); memcpy(q->Dp, Dp, sizeof(i64) * (size_t)(md + 1));
    q->Di = xmalloc(sizeof(i32) * (size_t)(Dp[md] ? Dp[md] : 1)); memcpy(q->Di, Di, sizeof(i32) * (size_t)Dp[md]);
    q->Dv = xmalloc(sizeof(double) * (size_t)(Dp[md] ? Dp[md] : 1)); memcpy(q->Dv, Dv, sizeof(double) * (size_t)Dp[md]);
    q->Ds = xmalloc(sizeof(double) * (size_t)(md ? md : 1)); memcpy(q->Ds, Ds, sizeof(double) * (size_t)md);
    /* tril(H + J_d^T D_s J_d) by triplets (row >= col), duplicates summed in
     * a fixed order, rows sorted */
    i64 cnt = Hp[n];
    for (i64 i = 0; i < md; i++) { i64 k = Dp[i + 1] - Dp[i]; cnt += k * (k + 1) / 2; }
    trip *t = xmalloc(sizeof(trip) * (size_t)(cnt ? cnt : 1));
    i64 z = 0;
    for (i64 i = 0; i < n; i++)
        for (i64 p = Hp[i]; p < Hp[i + 1]; p++) { t[z].row = Hi[p]; t[z].col = i; t[z].v = Hx[p]; t[z].seq = z; z++; }
    for (i64 i = 0; i < md; i++)
        for (i64 a = Dp[i]; a < Dp[i + 1]; a++)
            for (i64 b = Dp[i]; b < Dp[i + 1]; b++) {
                if (Di[a] < Di[b]) continue;
                /* stored as (row = larger index, col = smaller): tril by rows below */
                t[z].row = Di[b]; t[z].col = Di[a]; t[z].v = Ds[i] * Dv[a] * Dv[b]; t[z].seq = z; z++;
            }
    /* trip_cmp sorts by col then row: here col holds the CSR row (larger
     * index) and row the CSR column */
    qsort(t, (size_t)z, sizeof(trip), trip_cmp);
    i64 *Tp = xcalloc((size_t)n + 1, sizeof(i64));
    i32 *Ti = xmalloc(sizeof(i32) * (size_t)(z ? z : 1));
    double *Tx = xmalloc(sizeof(double) * (size_t)(z ? z : 1));
    i64 nz = 0;
    for (i64 k = 0; k < z; k++) {
        if (nz > 0 && k > 0 && t[k - 1].col == t[k].col && Ti[nz - 1] == t[k].row) Tx[nz - 1] += t[k].v;
        else { Ti[nz] = (i32)t[k].row; Tx[nz] = t[k].v; Tp[t[k].col + 1]++; nz++; }
    }
    for (i64 i = 0; i < n; i++) Tp[i + 1] += Tp[i];
    free(t);
    q->two = orc_new(n, m, Tp, Ti, Tx, Dx, Jp, Ji, Jx, delta, gamma);
    free(Tp); free(Ti); free(Tx);
    return q;
}

void orc4_free(orc4 *q) {
    if (!q) return;
    orc_free(q->two);
    free(q->Hp); free(q->Hi); free(q->Hx); free(q->Dp); free(q->Di); free(q->Dv); free(q->Ds);
    free(q);
}

orc *orc4_two(orc4 *q) { return q->two; }

/* g = r - K4 z, plain FP64, row by row */
static void res4(const orc4 *q, const double *rx, const double *rs, const double *ry, const double *ryd,
                 const double *x, const double *sv, const double *y, const double *yd,
                 double *gx, double *gs, double *gy, double *gyd) {
    const orc *s = q->two;
    i64 n = q->n, m = q->m, md = q->md;
    for (i64 i = 0; i < n; i++) gx[i] = rx[i] - (s->Dx[i] + s->delta) * x[i];
    for (i64 i = 0; i < n; i++)
        for (i64 p = q->Hp[i]; p < q->Hp[i + 1]; p++) {
            i64 j = q->Hi[p];
            gx[i] -= q->Hx[p] * x[j];
            if (j != i) gx[j] -= q->Hx[p] * x[i];
        }
    for (i64 k = 0; k < m; k++) {
        double jx = 0.0;
        for (i64 p = s->Jp[k]; p < s->Jp[k + 1]; p++) { jx += s->Jx[p] * x[s->Ji[p]]; gx[s->Ji[p]] -= s->Jx[p] * y[k]; }
        gy[k] = ry[k] - jx;
    }
    for (i64 k = 0; k < md; k++) {
        double dxk = 0.0;
        for (i64 p = q->Dp[k]; p < q->Dp[k + 1]; p++) { dxk += q->Dv[p] * x[q->Di[p]]; gx[q->Di[p]] -= q->Dv[p] * yd[k]; }
        gyd[k] = ryd[k] - (dxk - sv[k]);
        gs[k] = rs[k] - (q->Ds[k] * sv[k] - yd[k]);
    }
}

/* ||K4||_inf */
static double norm4(const orc4 *q) {
    const orc *s = q->two;
    i64 n = q->n, m = q->m, md = q->md;
    double *r = xcalloc((size_t)(n + md + m + md ? n + md + m + md : 1), sizeof(double));
    for (i64 i = 0; i < n; i++) {
        int has = 0;
        for (i64 p = q->Hp[i]; p < q->Hp[i + 1]; p++) {
            i64 j = q->Hi[p];
            if (j == i) { r[i] += fabs(q->Hx[p] + s->Dx[i] + s->delta); has = 1; }
            else { r[i] += fabs(q->Hx[p]); r[j] += fabs(q->Hx[p]); }
        }
        if (!has) r[i] += fabs(s->Dx[i] + s->delta);
    }
    for (i64 k = 0; k < m; k++)
        for (i64 p = s->Jp[k]; p < s->Jp[k + 1]; p++) { r[s->Ji[p]] += fabs(s->Jx[p]); r[n + md + k] += fabs(s->Jx[p]); }
    for (i64 k = 0; k < md; k++) {
        for (i64 p = q->Dp[k]; p < q->Dp[k + 1]; p++) { r[q->Di[p]] += fabs(q->Dv[p]); r[n + md + m + k] += fabs(q->Dv[p]); }
        r[n + k] += fabs(q->Ds[k]) + 1.0;
        r[n + md + m + k] += 1.0;
    }
    double mx = 0.0;
    for (i64 i = 0; i < n + md + m + md; i++) if (r[i] > mx) mx = r[i];
    free(r);
    return mx;
}

/* Solve K4 z = r: each step forms g = r - K4 z, reduces it to the 2x2
 * right-hand side r_x = g_x + J_d^T (D_s g_yd + g_s), r_y = g_y, solves the
 * 2x2 system by the hybrid method (with its own refinement to kkt_tol on the
 * 2x2 residual), recovers e_s = J_d e_x - g_yd, e_yd = D_s e_s - g_s and adds
 * e to z, while RR4 = ||g|| / ||r|| > kkt_tol and RR4 halves (at most
 * max_refine + 1 steps). The 2x2 system must be factored. out: [0] RR4,
 * [1] BE4 (||K4||_inf for ||K4||_2, Sec. 5.1), [2] steps, [3] total CG
 * iterations, [4] status (0 ok, 2 breakdown, 3 not converged). */
void orc4_solve(orc4 *q, const orc_opts *o, const double *rx, const double *rs, const double *ry, const double *ryd,
                double *x, double *sv, double *y, double *yd, double *out) {
    i64 n = q->n, m = q->m, md = q->md;
    double *gx = xmalloc(sizeof(double) * (size_t)(n ? n : 1)), *gs = xmalloc(sizeof(double) * (size_t)(md ? md : 1));
    double *gy = xmalloc(sizeof(double) * (size_t)(m ? m : 1)), *gyd = xmalloc(sizeof(double) * (size_t)(md ? md : 1));
    double *ex = xmalloc(sizeof(double) * (size_t)(n ? n : 1)), *ey = xmalloc(sizeof(double) * (size_t)(m ? m : 1));
    double *r2x = xmalloc(sizeof(double) * (size_t)(n ? n : 1)), *t = xmalloc(sizeof(double) * (size_t)(md ? md : 1));
    for (i64 i = 0; i < n; i++) x[i] = 0.0;
    for (i64 i = 0; i < m; i++) y[i] = 0.0;
    for (i64 i = 0; i < md; i++) { sv[i] = 0.0; yd[i] = 0.0; }
    double rn = sqrt(dot(rx, rx, n) + dot(rs, rs, md) + dot(ry, ry, m) + dot(ryd, ryd, md));
    i64 max_ref = o->max_refine > 0 ? o->max_refine : 10;
    double rr = rn > 0 ? 1.0 : 0.0, best = INFINITY;
    i64 steps = 0, cg = 0;
    int status = 3;
    orc_report rep;
    for (;;) {
        res4(q, rx, rs, ry, ryd, x, sv, y, yd, gx, gs, gy, gyd);
        rr = rn > 0 ? sqrt(dot(gx, gx, n) + dot(gs, gs, md) + dot(gy, gy, m) + dot(gyd, gyd, md)) / rn : 0.0;
        if (rr <= o->kkt_tol) { status = 0; break; }
        if (steps > max_ref || (steps >= 2 && !(rr < 0.5 * best))) break;
        if (rr < best) best = rr;
        for (i64 k = 0; k < md; k++) t[k] = q->Ds[k] * gyd[k] + gs[k];
        for (i64 i = 0; i < n; i++) r2x[i] = gx[i];
        for (i64 k = 0; k < md; k++)
            for (i64 p = q->Dp[k]; p < q->Dp[k + 1]; p++) r2x[q->Di[p]] += q->Dv[p] * t[k];
        orc_solve(q->two, o, r2x, gy, ex, ey, &rep);
        for (i64 c = 0; c < rep.passes; c++) cg += rep.cg_iters[c];
        steps++;
        if (rep.status == 2) { status = 2; }
        for (i64 i = 0; i < n; i++) x[i] += ex[i];
        for (i64 i = 0; i < m; i++) y[i] += ey[i];
        for (i64 k = 0; k < md; k++) {
            double jx = 0.0;
            for (i64 p = q->Dp[k]; p < q->Dp[k + 1]; p++) jx += q->Dv[p] * ex[q->Di[p]];
            double es = jx - gyd[k];
            sv[k] += es;
            yd[k] += q->Ds[k] * es - gs[k];
        }
        if (status == 2) {
            res4(q, rx, rs, ry, ryd, x, sv, y, yd, gx, gs, gy, gyd);
            rr = rn > 0 ? sqrt(dot(gx, gx, n) + dot(gs, gs, md) + dot(gy, gy, m) + dot(gyd, gyd, md)) / rn : 0.0;
            break;
        }
    }
    double zn = sqrt(dot(x, x, n) + dot(sv, sv, md) + dot(y, y, m) + dot(yd, yd, md));
    double gn = rr * (rn > 0 ? rn : 1.0);
    out[0] = rr;
    out[1] = gn / (norm4(q) * zn + rn);
    out[2] = (double)steps;
    out[3] = (double)cg;
    out[4] = (double)status;
    free(gx); free(gs); free(gy); free(gyd); free(ex); free(ey); free(r2x); free(t);
}

/* RR4, BE4 of a given z (plain FP64 residual) */
void orc4_metrics(const orc4 *q, const double *rx, const double *rs, const double *ry, const double *ryd,
                  const double *x, const double *sv, const double *y, const double *yd, double *out2) {
    i64 n = q->n, m = q->m, md = q->md;
    double *gx = xmalloc(sizeof(double) * (size_t)(n ? n : 1)), *gs = xmalloc(sizeof(double) * (size_t)(md ? md : 1));
    double *gy = xmalloc(sizeof(double) * (size_t)(m ? m : 1)), *gyd = xmalloc(sizeof(double) * (size_t)(md ? md : 1));
    res4(q, rx, rs, ry, ryd, x, sv, y, yd, gx, gs, gy, gyd);
    double rn = sqrt(dot(rx, rx, n) + dot(rs, rs, md) + dot(ry, ry, m) + dot(ryd, ryd, md));
    double gn = sqrt(dot(gx, gx, n) + dot(gs, gs, md) + dot(gy, gy, m) + dot(gyd, gyd, md));
    double zn = sqrt(dot(x, x, n) + dot(sv, sv, md) + dot(y, y, m) + dot(yd, yd, md));
    out2[0] = rn > 0 ? gn / rn : gn;
    out2[1] = gn / (norm4(q) * zn + rn);
    free(gx); free(gs); free(gy); free(gyd);
}
