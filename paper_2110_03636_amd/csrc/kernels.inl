// Device kernels (gfx950), included by the library translation unit: assembly of H_gamma into supernodal storage,
// multifrontal supernodal Cholesky, supernodal triangular solves, SpMV with
// J and J^T, CG vector updates with deterministic reductions, and the FP64
// KKT residual. Templated on the factor/solve precision T (float or double);
// every reduction and every CG scalar is FP64.
#include "kernels.hpp"

#include <cfloat>
#include <climits>

namespace hkkt {

// Solve-phase kernels run over a list of instance ids (the instances still
// active); grid index k maps to instance ids[k] (ids null: k itself).
__device__ __forceinline__ int inst_of(const int* ids, int k) { return ids ? ids[k] : k; }

// Group member of permuted variable i (0 for a single pattern). Scalars of
// member k of batch entry b (delta, gamma, CG state, failure column, norms)
// sit at index b * G + k.
__device__ __forceinline__ int mem_x(const SymView& S, i64 i) { return S.G > 1 ? S.xp_mem[i] : 0; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
    return v;
}

// Value of lane jl (the same in all active lanes) in every lane (v_readlane).
__device__ __forceinline__ float lane_read(float v, int jl) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), __builtin_amdgcn_readfirstlane(jl)));
}
__device__ __forceinline__ double lane_read(double v, int jl) {
    const long long u = __double_as_longlong(v);
    const int l = __builtin_amdgcn_readfirstlane(jl);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Block sum; the result is valid in thread 0. `sh` holds kBlock/kWave doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x / kWave); i++) r += sh[i];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// utility
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* __restrict__ p, i64 n, T v) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] = v;
}

template <typename TI, typename TO>
__global__ void k_cast(const TI* __restrict__ in, TO* __restrict__ out, i64 len, const int* ids,
                       const CGState* st) {
    const int b = inst_of(ids, blockIdx.y);
    if (st && st[b].done) return;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (i64)gridDim.x * blockDim.x)
        out[(i64)b * len + i] = (TO)in[(i64)b * len + i];
}

// permuted gather: out[b][k] = in[b][perm[k]]
__global__ void k_perm_gather(const i32* __restrict__ perm, const double* __restrict__ in, double* __restrict__ out,
                              i64 n) {
    const int b = blockIdx.y;
    for (i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x)
        out[(i64)b * n + k] = in[(i64)b * n + perm[k]];
}

// permuted scatter: out[b][perm[k]] = in[b][k]
__global__ void k_perm_scatter(const i32* __restrict__ perm, const double* __restrict__ in, double* __restrict__ out,
                               i64 n) {
    const int b = blockIdx.y;
    for (i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x)
        out[(i64)b * n + perm[k]] = in[(i64)b * n + k];
}

// values of J^T (JT order), full symmetric H (permuted) and D_x (permuted)
__global__ void k_gather_vals(SymView S, const double* __restrict__ H, const double* __restrict__ J,
                              const double* __restrict__ Dx, double* __restrict__ JT, double* __restrict__ HF,
                              double* __restrict__ Dxp) {
    const int b = blockIdx.y;
    const i64 stride = (i64)gridDim.x * blockDim.x;
    for (i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x; k < S.nnzJ; k += stride)
        JT[(i64)b * S.nnzJ + k] = J[(i64)b * S.nnzJ + S.JT_src[k]];
    for (i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x; k < S.nnzHF; k += stride)
        HF[(i64)b * S.nnzHF + k] = H[(i64)b * S.nnzH + S.HF_src[k]];
    for (i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x; k < S.n; k += stride)
        Dxp[(i64)b * S.n + k] = Dx[(i64)b * S.n + S.perm[k]];
}

// ---------------------------------------------------------------------------
// symmetrized Ruiz scaling of K = [H + D_x + delta I, J^T; J, 0] (Sec. 4.1):
// sc per instance holds d over [x rows in the permuted order ; J rows]. One
// sweep: rm_i = max_j |(D K D)_ij| (k_ruiz_rows), then d_i /= sqrt(rm_i)
// (k_ruiz_apply, rows that are all zero keep their d).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_ruiz_rows(SymView S, ValView V, const double* __restrict__ sc,
                                                      double* __restrict__ rm) {
    // four lanes per row, each taking every fourth entry of the row's runs
    // (consecutive lanes read consecutive entries), then a max over the four
    // lanes (and a sum for the diagonal, which one lane holds): the same
    // products as one thread per row, so the same maxima
    const int b = blockIdx.y;
    const i64 nm = S.n + S.m;
    const double* d = sc + (i64)b * nm;
    const int l4 = threadIdx.x & 3;
    const i64 step = ((i64)gridDim.x * blockDim.x) >> 2;
    for (i64 i = ((i64)blockIdx.x * blockDim.x + threadIdx.x) >> 2; i < nm; i += step) {
        double a = 0.0;
        if (i < S.n) {
            const double* HF = V.HF + (i64)b * S.nnzHF;
            const double* JT = V.JT + (i64)b * S.nnzJ;
            const int k = S.G > 1 ? S.xp_mem[i] : 0;
            double dg = l4 == 0 ? V.Dxp[(i64)b * S.n + i] + V.delta[(i64)b * S.G + k] : 0.0;
            const double di = d[i];
            for (i64 q = S.HF_rowptr[i] + l4; q < S.HF_rowptr[i + 1]; q += 4) {
                if (S.HF_col[q] == i) dg += HF[q];
                else a = fmax(a, fabs(HF[q]) * di * d[S.HF_col[q]]);
            }
            dg += __shfl_xor(dg, 1, 4);
            dg += __shfl_xor(dg, 2, 4);
            a = fmax(a, fabs(dg) * di * di);
            for (i64 q = S.JT_rowptr[i] + l4; q < S.JT_rowptr[i + 1]; q += 4)
                a = fmax(a, fabs(JT[q]) * di * d[S.n + S.JT_col[q]]);
        } else {
            const double* J = V.J + (i64)b * S.nnzJ;
            const i64 r = i - S.n;
            const double dr = d[i];
            for (i64 q = S.J_rowptr[r] + l4; q < S.J_rowptr[r + 1]; q += 4)
                a = fmax(a, fabs(J[q]) * dr * d[S.J_colp[q]]);
        }
        a = fmax(a, __shfl_xor(a, 1, 4));
        a = fmax(a, __shfl_xor(a, 2, 4));
        if (l4 == 0) rm[(i64)b * nm + i] = a;
    }
}

__global__ void k_ruiz_apply(i64 len, double* __restrict__ sc, const double* __restrict__ rm) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (i64)gridDim.x * blockDim.x)
        if (rm[i] > 0.0) sc[i] /= sqrt(rm[i]);
}

// Values of the scaled system D K D: H' = D1 H D1 (full permuted HF', and
// tril H' in the caller's order by scattering HF' through HF_src: both
// triangle entries of a pair carry the same value), J' = D2 J D1, J'^T, and
// the diagonal D_x' = d1^2 (D_x + delta) (delta folded in; the scaled
// system's delta is 0), permuted and in the caller's order.
__global__ __launch_bounds__(kBlock) void k_scale_vals(SymView S, ValView V, const double* __restrict__ sc,
                                                       double* __restrict__ Hs, double* __restrict__ Js,
                                                       double* __restrict__ JTs, double* __restrict__ HFs,
                                                       double* __restrict__ Dxps, double* __restrict__ Dxs) {
    // four lanes per row, every fourth entry each (as in k_ruiz_rows)
    const int b = blockIdx.y;
    const i64 nm = S.n + S.m;
    const double* d = sc + (i64)b * nm;
    const int l4 = threadIdx.x & 3;
    const i64 step = ((i64)gridDim.x * blockDim.x) >> 2;
    for (i64 i = ((i64)blockIdx.x * blockDim.x + threadIdx.x) >> 2; i < nm; i += step) {
        if (i < S.n) {
            const double di = d[i];
            for (i64 q = S.HF_rowptr[i] + l4; q < S.HF_rowptr[i + 1]; q += 4) {
                const double v = V.HF[(i64)b * S.nnzHF + q] * di * d[S.HF_col[q]];
                HFs[(i64)b * S.nnzHF + q] = v;
                Hs[(i64)b * S.nnzH + S.HF_src[q]] = v;
            }
            for (i64 q = S.JT_rowptr[i] + l4; q < S.JT_rowptr[i + 1]; q += 4)
                JTs[(i64)b * S.nnzJ + q] = V.JT[(i64)b * S.nnzJ + q] * di * d[S.n + S.JT_col[q]];
            if (l4 == 0) {
                const int k = S.G > 1 ? S.xp_mem[i] : 0;
                const double v = di * di * (V.Dxp[(i64)b * S.n + i] + V.delta[(i64)b * S.G + k]);
                Dxps[(i64)b * S.n + i] = v;
                Dxs[(i64)b * S.n + S.perm[i]] = v;
            }
        } else {
            const i64 r = i - S.n;
            const double dr = d[i];
            for (i64 q = S.J_rowptr[r] + l4; q < S.J_rowptr[r + 1]; q += 4)
                Js[(i64)b * S.nnzJ + q] = V.J[(i64)b * S.nnzJ + q] * dr * d[S.J_colp[q]];
        }
    }
}

// x[b][i] *= d[b][i] (i < n, permuted order) and y[b][r] *= d[b][n + r] for
// the instances listed in ids (all when null): a vector pair into or out of
// the scaled system
__global__ void k_scale_pair(const double* __restrict__ sc, i64 n, i64 m, double* __restrict__ x,
                             double* __restrict__ y, const int* ids) {
    const int b = inst_of(ids, blockIdx.y);
    const double* d = sc + (i64)b * (n + m);
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n + m; i += (i64)gridDim.x * blockDim.x) {
        if (i < n) x[(i64)b * n + i] *= d[i];
        else y[(i64)b * m + (i - n)] *= d[i];
    }
}

// ---------------------------------------------------------------------------
// the 4x4 system of Sec. 3 (eq. linsys4x4) around the 2x2 solver, in the
// caller's variable order, plain FP64
// ---------------------------------------------------------------------------
// out[b][i] = (acc ? out[b][i] : 0) + alpha * sum_k vals[b][src[k]] x[b][col[k]]
// over row i of a CSR pattern whose values are gathered through src (null:
// the k-th value)
__global__ void k_spmv_src(i64 nrow, const i64* __restrict__ rowptr, const i32* __restrict__ col,
                           const i64* __restrict__ src, const double* __restrict__ vals, i64 nnz,
                           const double* __restrict__ x, i64 ncol, double* __restrict__ out, double alpha, int acc) {
    const int b = blockIdx.y;
    const double* v = vals + (i64)b * nnz;
    const double* xb = x + (i64)b * ncol;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < nrow; i += (i64)gridDim.x * blockDim.x) {
        double a = 0.0;
        for (i64 k = rowptr[i]; k < rowptr[i + 1]; k++) a += v[src ? src[k] : k] * xb[col[k]];
        out[(i64)b * nrow + i] = (acc ? out[(i64)b * nrow + i] : 0.0) + alpha * a;
    }
}

// Htilde's H part, H + J_d^T D_s J_d, on the combined pattern: entry e takes
// H[h_src[e]] (if any) plus D_s[k] J_d[a] J_d[b] for its pairs, in a fixed
// order
__global__ void k_htilde(i64 nnz, const i64* __restrict__ h_src, const i64* __restrict__ pptr,
                         const i32* __restrict__ prow, const i64* __restrict__ pa, const i64* __restrict__ pb,
                         const double* __restrict__ H, i64 nnzH, const double* __restrict__ Jd, i64 nnzJd,
                         const double* __restrict__ Ds, i64 md, double* __restrict__ Ht) {
    const int b = blockIdx.y;
    for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (i64)gridDim.x * blockDim.x) {
        double v = h_src[e] >= 0 ? H[(i64)b * nnzH + h_src[e]] : 0.0;
        for (i64 p = pptr[e]; p < pptr[e + 1]; p++)
            v += Ds[(i64)b * md + prow[p]] * Jd[(i64)b * nnzJd + pa[p]] * Jd[(i64)b * nnzJd + pb[p]];
        Ht[(i64)b * nnz + e] = v;
    }
}

// the 4x4 residual from the products: tx = H x + J^T y + J_d^T y_d, jx = J x,
// dx = J_d x (all already formed):
//   g_x = r_x - tx - (D_x + delta) x,  g_y = r_y - jx,
//   g_yd = r_yd - (dx - s),             g_s = r_s - (D_s s - y_d)
// and the reduced right-hand side parts t = D_s g_yd + g_s
__global__ void k_res4(i64 n, i64 m, i64 md, const double* __restrict__ Dx, const double* __restrict__ delta,
                       const double* __restrict__ Ds, const double* __restrict__ rx, const double* __restrict__ rs,
                       const double* __restrict__ ry, const double* __restrict__ ryd, const double* __restrict__ x,
                       const double* __restrict__ s, const double* __restrict__ yd, const double* __restrict__ tx,
                       const double* __restrict__ jx, const double* __restrict__ dx, double* __restrict__ gx,
                       double* __restrict__ gs, double* __restrict__ gy, double* __restrict__ gyd,
                       double* __restrict__ t) {
    const int b = blockIdx.y;
    const i64 tot = n + m + md;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (i64)gridDim.x * blockDim.x) {
        if (i < n) {
            const i64 q = (i64)b * n + i;
            gx[q] = rx[q] - tx[q] - (Dx[q] + delta[b]) * x[q];
        } else if (i < n + m) {
            const i64 q = (i64)b * m + (i - n);
            gy[q] = ry[q] - jx[q];
        } else {
            const i64 q = (i64)b * md + (i - n - m);
            const double a = ryd[q] - (dx[q] - s[q]);
            const double c = rs[q] - (Ds[q] * s[q] - yd[q]);
            gyd[q] = a;
            gs[q] = c;
            t[q] = Ds[q] * a + c;
        }
    }
}

// after the 2x2 correction (e_x, e_y) of the active instances: x += e_x,
// y += e_y, e_s = J_d e_x - g_yd (jde = J_d e_x formed), s += e_s,
// y_d += D_s e_s - g_s
__global__ void k_recover4(i64 n, i64 m, i64 md, const int* __restrict__ active, const double* __restrict__ Ds,
                           const double* __restrict__ ex, const double* __restrict__ ey,
                           const double* __restrict__ jde, const double* __restrict__ gs,
                           const double* __restrict__ gyd, double* __restrict__ x, double* __restrict__ y,
                           double* __restrict__ s, double* __restrict__ yd) {
    const int b = blockIdx.y;
    if (!active[b]) return;
    const i64 tot = n + m + md;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (i64)gridDim.x * blockDim.x) {
        if (i < n) x[(i64)b * n + i] += ex[(i64)b * n + i];
        else if (i < n + m) y[(i64)b * m + (i - n)] += ey[(i64)b * m + (i - n)];
        else {
            const i64 q = (i64)b * md + (i - n - m);
            const double es = jde[q] - gyd[q];
            s[q] += es;
            yd[q] += Ds[q] * es - gs[q];
        }
    }
}

// per instance (one block): out[b] = sum of squares of the four vectors
// (lengths n, md, m, md; a null vector counts as zero)
__global__ __launch_bounds__(kBlock) void k_sumsq4(i64 n, i64 md, i64 m, const double* __restrict__ a,
                                                   const double* __restrict__ c, const double* __restrict__ d,
                                                   const double* __restrict__ e, double* __restrict__ out) {
    __shared__ double sh[kBlock / kWave];
    const int b = blockIdx.x;
    double acc = 0.0;
    for (i64 i = threadIdx.x; i < n; i += blockDim.x) { const double v = a[(i64)b * n + i]; acc += v * v; }
    for (i64 i = threadIdx.x; i < md; i += blockDim.x) {
        const double v = c[(i64)b * md + i], w = e[(i64)b * md + i];
        acc += v * v + w * w;
    }
    for (i64 i = threadIdx.x; i < m; i += blockDim.x) { const double v = d[(i64)b * m + i]; acc += v * v; }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) out[b] = acc;
}

// per instance (one block): ||K4||_inf from the row sums: x rows |H| (full
// pattern) + |D_x + delta| + |J^T| + |J_d^T|; s rows |D_s| + 1; y rows |J|;
// y_d rows |J_d| + 1
__global__ __launch_bounds__(kBlock) void k_norm4(i64 n, i64 m, i64 md, const i64* __restrict__ hf_ptr,
                                                  const i32* __restrict__ hf_col, const i64* __restrict__ hf_src,
                                                  const double* __restrict__ H, i64 nnzH,
                                                  const double* __restrict__ Dx, const double* __restrict__ delta,
                                                  const i64* __restrict__ jt_ptr, const i64* __restrict__ jt_src,
                                                  const double* __restrict__ J, i64 nnzJ,
                                                  const i64* __restrict__ dt_ptr, const i64* __restrict__ dt_src,
                                                  const double* __restrict__ Jd, i64 nnzJd,
                                                  const i64* __restrict__ j_ptr, const i64* __restrict__ d_ptr,
                                                  const double* __restrict__ Ds, double* __restrict__ out) {
    __shared__ double sh[kBlock / kWave];
    const int b = blockIdx.x;
    double mx = 0.0;
    for (i64 i = threadIdx.x; i < n; i += blockDim.x) {
        double r = 0.0, dg = Dx[(i64)b * n + i] + delta[b];
        for (i64 k = hf_ptr[i]; k < hf_ptr[i + 1]; k++) {
            const double v = H[(i64)b * nnzH + hf_src[k]];
            if (hf_col[k] == i) dg += v;
            else r += fabs(v);
        }
        r += fabs(dg);
        for (i64 k = jt_ptr[i]; k < jt_ptr[i + 1]; k++) r += fabs(J[(i64)b * nnzJ + jt_src[k]]);
        for (i64 k = dt_ptr[i]; k < dt_ptr[i + 1]; k++) r += fabs(Jd[(i64)b * nnzJd + dt_src[k]]);
        mx = fmax(mx, r);
    }
    for (i64 i = threadIdx.x; i < md; i += blockDim.x) {
        mx = fmax(mx, fabs(Ds[(i64)b * md + i]) + 1.0);
        double r = 1.0;
        for (i64 k = d_ptr[i]; k < d_ptr[i + 1]; k++) r += fabs(Jd[(i64)b * nnzJd + k]);
        mx = fmax(mx, r);
    }
    for (i64 i = threadIdx.x; i < m; i += blockDim.x) {
        double r = 0.0;
        for (i64 k = j_ptr[i]; k < j_ptr[i + 1]; k++) r += fabs(J[(i64)b * nnzJ + k]);
        mx = fmax(mx, r);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) mx = fmax(mx, __shfl_down(mx, o, kWave));
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int t = 0; t < (int)(blockDim.x / kWave); t++) r = fmax(r, sh[t]);
        out[b] = r;
    }
}

// dst[i][0:len) = src[idx[i]][0:len) (gather of batch entries; grid.y = entry)
__global__ void k_gather_inst(const double* __restrict__ src, double* __restrict__ dst, i64 len,
                              const int* __restrict__ idx) {
    const i64 so = (i64)idx[blockIdx.y] * len, d0 = (i64)blockIdx.y * len;
    for (i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += (i64)gridDim.x * blockDim.x)
        dst[d0 + k] = src[so + k];
}

// dst[didx[i]][0:len) = src[sidx[i]][0:len) (rows of batch entries)
__global__ void k_copy_rows(const double* __restrict__ src, double* __restrict__ dst, i64 len,
                            const int* __restrict__ sidx, const int* __restrict__ didx) {
    const i64 s0 = (i64)sidx[blockIdx.y] * len, d0 = (i64)didx[blockIdx.y] * len;
    for (i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += (i64)gridDim.x * blockDim.x)
        dst[d0 + k] = src[s0 + k];
}

// ---------------------------------------------------------------------------
// assembly: H_gamma = tril(H) + diag(D_x + delta) + gamma * tril(J^T J)
// (Sec. 3 and eq. eq:gamma), one thread per entry of tril(P H_gamma P^T),
// summed in FP64 in a fixed order and written into the supernodal panels.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_assemble(SymView S, ValView V, T* __restrict__ L, const int* active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const double* H = V.H + (i64)b * S.nnzH;
    const double* J = V.J + (i64)b * S.nnzJ;
    const double* gam = V.gamma + (i64)b * S.G;
    const double* del = V.delta + (i64)b * S.G;
    T* Lb = L + (i64)b * S.Lsize;
    for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < S.nnzA; e += (i64)gridDim.x * blockDim.x) {
        const int k = S.G > 1 ? S.a_mem[e] : 0;
        const double g = gam[k], dl = del[k];
        double v = 0.0;
        const i32 h = S.a_h[e];
        if (h >= 0) v += H[h];
        const i32 d = S.a_d[e];
        if (d >= 0) v += V.Dx[(i64)b * S.n + d] + dl;
        for (i64 p = S.a_pptr[e]; p < S.a_pptr[e + 1]; p++) v += g * J[S.a_pa[p]] * J[S.a_pb[p]];
        Lb[S.a_dst[e]] = (T)v;
    }
}

// ---------------------------------------------------------------------------
// multifrontal supernodal Cholesky
//
// Front of supernode s: F (nr x nr, lower) = [panel of s (assembled entries of
// its w columns) | zero update block], plus the extend-add of every child's
// contribution block. Partial factorization of the first w columns:
//   L11 = chol(F11), L21 = F21 L11^{-T}, CB = F22 - L21 L21^T.
// Right-looking by columns with a single barrier per column: step k scales
// column k-1 (with the pivot read in step k-1) while it applies the rank-1
// update of column k to the trailing matrix; the two phases touch disjoint
// columns. A pivot <= 0 or not finite records the smallest failing column.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ bool pivot_ok(T d) {
    return d > T(0) && d <= (T)(sizeof(T) == 8 ? DBL_MAX : FLT_MAX);
}

// adiag (may be null): the FP64 diagonal of H_gamma per (instance, pivot);
// a pivot below ptol times it clears the instance's entry of act_w (the
// active array this factorization reads), so the instance's later fronts
// are skipped (the instance is refactored in FP64)
template <typename T>
__device__ __forceinline__ void pivot_stop(const double* adiag, double ptol, int* act_w, const SymView& S, int b,
                                           i64 col, T d) {
    if (adiag && !((double)d >= ptol * adiag[(i64)b * S.n + col])) act_w[b] = 0;
}

// (column, row) of the flat column-major index idx = col * len + row of a
// len x len block, stepped by the block size without a division per step:
// the same elements in the same order as idx / len, idx % len.
struct SqIdx {
    int col, row, dcol, drow, len;
    __device__ __forceinline__ SqIdx(int idx, int step, int n) : len(n) {
        col = idx / n;
        row = idx - col * n;
        dcol = step / n;
        drow = step - dcol * n;
    }
    __device__ __forceinline__ void next() {
        row += drow;
        col += dcol;
        if (row >= len) {
            row -= len;
            col++;
        }
    }
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_front_lds(SymView S, const i32* __restrict__ list, T* __restrict__ L,
                                                      T* __restrict__ CB, int* __restrict__ fail, const int* active,
                                                      const double* adiag, double ptol, int* act_w) {
    extern __shared__ double smem_d[];
    T* F = reinterpret_cast<T*>(smem_d);
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const i32 s = list[blockIdx.x];
    const i32 f = S.sn_first[s];
    const int w = S.sn_first[s + 1] - f;
    const int nr = (int)(S.sn_rowptr[s + 1] - S.sn_rowptr[s]);
    const int nc = nr - w;
    T* Lb = L + (i64)b * S.Lsize + S.sn_lptr[s];
    const int nn = nr * nr;
    for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) F[idx] = idx < nr * w ? Lb[idx] : T(0);
    __syncthreads();
    for (int q = S.child_ptr[s]; q < S.child_ptr[s + 1]; q++) {
        const i32 c = S.child_list[q];
        const int wc = S.sn_first[c + 1] - S.sn_first[c];
        const int ncc = (int)(S.sn_rowptr[c + 1] - S.sn_rowptr[c]) - wc;
        const i32* rel = S.relmap + S.sn_uvptr[c];
        const T* C = CB + (i64)b * S.CBsize + S.sn_cbptr[c];
        if (ncc > 0) {
            SqIdx t(threadIdx.x, blockDim.x, ncc);
            for (int idx = threadIdx.x; idx < ncc * ncc; idx += blockDim.x, t.next())
                if (t.row >= t.col) F[rel[t.col] * nr + rel[t.row]] += C[idx];
        }
        __syncthreads();
    }
    T dprev = T(1);
    for (int k = 0; k <= w; k++) {
        const T dk = k < w ? F[k * nr + k] : T(1);
        if (k > 0) {
            const int kk = k - 1;
            const T sq = sqrt(dprev), inv = T(1) / sq;
            for (int i = kk + threadIdx.x; i < nr; i += blockDim.x) F[kk * nr + i] = i == kk ? sq : F[kk * nr + i] * inv;
        }
        if (k < w) {
            if (threadIdx.x == 0 && !pivot_ok(dk)) atomicMin(&fail[b * S.G + (S.G > 1 ? S.sn_mem[s] : 0)], f + k);
            if (threadIdx.x == 0) pivot_stop(adiag, ptol, act_w, S, b, f + k, dk);
            const T invd = T(1) / dk;
            const int len = nr - k - 1;
            if (len > 0) {
                SqIdx t(threadIdx.x, blockDim.x, len);
                for (int idx = threadIdx.x; idx < len * len; idx += blockDim.x, t.next()) {
                    if (t.row >= t.col) {
                        const int i = k + 1 + t.row, j = k + 1 + t.col;
                        F[j * nr + i] -= F[k * nr + i] * F[k * nr + j] * invd;
                    }
                }
            }
        }
        dprev = dk;
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < nr * w; idx += blockDim.x) Lb[idx] = F[idx];
    T* C = CB + (i64)b * S.CBsize + S.sn_cbptr[s];
    if (nc > 0) {
        SqIdx t(threadIdx.x, blockDim.x, nc);
        for (int idx = threadIdx.x; idx < nc * nc; idx += blockDim.x, t.next())
            if (t.row >= t.col) C[idx] = F[(w + t.col) * nr + w + t.row];
    }
}

// Same partial factorization for fronts too large for LDS: the front lives in
// its panel (L storage) and its contribution block (CB workspace).
template <typename T>
struct FrontRef {
    T* P;   // panel nr x w
    T* C;   // contribution block nc x nc
    int nr, w, nc;
    __device__ __forceinline__ T& at(int i, int j) const {
        return j < w ? P[(i64)j * nr + i] : C[(i64)(j - w) * nc + (i - w)];
    }
};


// ---------------------------------------------------------------------------
// Blocked partial factorization of large fronts (above the LDS limit), one
// step per NB = 32 columns, all large fronts of a level and all instances in
// the same launches (grid.y = front, grid.z = instance):
//   k_big_zero    clear the fronts' contribution blocks
//   k_big_extend  add the children's contribution blocks (one child rank per
//                 launch, so two children never write one front at once)
//   k_big_ptrsm   Cholesky of the NB x NB diagonal block (one wavefront)
//                 and L21 = A21 L11^{-T}, one thread per row
//   k_big_update  SYRK/GEMM C -= L21 L21^T on 64 x 64 lower tiles, rank up to
//                 128: inside a 128-column block each panel first takes the
//                 block's earlier panels (left-looking strip), then one
//                 trailing update per block (right-looking, k_big_update2 on
//                 128 x 128 tiles)
//                 with MFMA (v_mfma_*_16x16x4: A[i][k] in lane i+16k,
//                 B[k][j] in lane j+16k; D[i][j] in lane j+16q, register r
//                 with i = 4q+r for f32 and i = q+4r for f64, as measured)
// ---------------------------------------------------------------------------
constexpr int kNB = 32;
constexpr int kTile = 64;

template <typename T>
__device__ __forceinline__ FrontRef<T> front_of(const SymView& S, i32 s, int b, T* L, T* CB) {
    FrontRef<T> F;
    const i32 f = S.sn_first[s];
    F.w = S.sn_first[s + 1] - f;
    F.nr = (int)(S.sn_rowptr[s + 1] - S.sn_rowptr[s]);
    F.nc = F.nr - F.w;
    F.P = L + (i64)b * S.Lsize + S.sn_lptr[s];
    F.C = CB + (i64)b * S.CBsize + S.sn_cbptr[s];
    return F;
}

template <typename T>
__global__ void k_big_zero(SymView S, const i32* __restrict__ fronts, T* __restrict__ CB, const int* active) {
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const i32 s = fronts[blockIdx.y];
    const i64 nc = (S.sn_rowptr[s + 1] - S.sn_rowptr[s]) - (S.sn_first[s + 1] - S.sn_first[s]);
    T* C = CB + (i64)b * S.CBsize + S.sn_cbptr[s];
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < nc * nc; i += (i64)gridDim.x * blockDim.x) C[i] = T(0);
}

// pairs[2q] = front, pairs[2q+1] = its child of the launch's rank. Work-group
// x takes kExtCols consecutive columns of the child's contribution block
// (lower triangle); its threads walk the rows, so the block is read in
// contiguous column segments and the front is written along the (sorted)
// row map.
constexpr int kExtCols = 4;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_big_extend(SymView S, const i32* __restrict__ pairs, T* __restrict__ L,
                                                       T* __restrict__ CB, const int* active) {
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const i32 s = pairs[2 * blockIdx.y], c = pairs[2 * blockIdx.y + 1];
    const int wc = S.sn_first[c + 1] - S.sn_first[c];
    const int ncc = (int)(S.sn_rowptr[c + 1] - S.sn_rowptr[c]) - wc;
    const int j0 = blockIdx.x * kExtCols;
    if (j0 >= ncc) return;
    const FrontRef<T> F = front_of<T>(S, s, b, L, CB);
    const i32* rel = S.relmap + S.sn_uvptr[c];
    const T* C = CB + (i64)b * S.CBsize + S.sn_cbptr[c];
    for (int j = j0; j < min(ncc, j0 + kExtCols); j++) {
        const int rj = rel[j];
        const T* cj = C + (i64)j * ncc;
        for (int i = j + threadIdx.x; i < ncc; i += blockDim.x) F.at(rel[i], rj) += cj[i];
    }
}

// POTRF and TRSM of one 32-column panel in one launch. Every work-group
// factors the NB x NB diagonal block in its first wavefront: lane i holds
// row i in registers, column k is scaled and its values broadcast with
// v_readlane (uniform lane index), no LDS and no barriers. It shares the
// factored block through LDS and solves L21 = A21 L11^{-T} for its rows
// below, one thread per row. The block is factored redundantly per
// work-group (a few microseconds of one wavefront) instead of by a launch
// of its own, identically in each (the same operations on the same values).
// Every work-group of a (front, instance) reads the unfactored block, so
// the factored one is stored by the last of them to finish: each counts
// itself in cnt[(instance, front slot)] after its reads have been consumed
// (its own stores done and fenced), and the one that completes the count
// stores the block and resets the counter to zero for the next panel.
// Work-group 0 reports a failed pivot.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_big_ptrsm(SymView S, const i32* __restrict__ fronts, int kb,
                                                      T* __restrict__ L, T* __restrict__ CB, int* __restrict__ fail,
                                                      int* __restrict__ cnt, const int* active, const double* adiag,
                                                      double ptol, int* act_w) {
    __shared__ T D[kNB][kNB + 1];
    __shared__ int last;
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const i32 s = fronts[blockIdx.y];
    const FrontRef<T> F = front_of<T>(S, s, b, L, CB);
    const int bw = min(kNB, F.w - kb);
    if (bw <= 0) return;
    const bool rows_here = kb + bw + (int)(blockIdx.x * blockDim.x) < F.nr;
    if (blockIdx.x > 0 && !rows_here) return;   // whole block past the front
    // work-groups of this (front, instance) that read the block: x = 0 and
    // every x with rows below
    const int below = F.nr - kb - bw;
    const int nwg = below > 0 ? (below + (int)blockDim.x - 1) / (int)blockDim.x : 1;
    if (threadIdx.x < kWave) {
        const int i = threadIdx.x;
        T r[kNB];
#pragma unroll
        for (int j = 0; j < kNB; j++) r[j] = (i < bw && j <= i) ? F.P[(i64)(kb + j) * F.nr + kb + i] : T(0);
        const i32 f = S.sn_first[s];
#pragma unroll
        for (int k = 0; k < kNB; k++) {
            if (k < bw) {
                const T d = lane_read(r[k], k);
                if (i == 0 && blockIdx.x == 0 && !pivot_ok(d))
                    atomicMin(&fail[b * S.G + (S.G > 1 ? S.sn_mem[s] : 0)], f + kb + k);
                if (i == 0 && blockIdx.x == 0) pivot_stop(adiag, ptol, act_w, S, b, f + kb + k, d);
                const T sq = sqrt(d), inv = T(1) / sq;
                r[k] = i == k ? sq : (i > k ? r[k] * inv : r[k]);
#pragma unroll
                for (int j = k + 1; j < kNB; j++) {
                    if (j < bw) {
                        const T ljk = lane_read(r[k], j);
                        if (i >= j) r[j] -= r[k] * ljk;
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kNB; j++)
            if (i < bw && j <= i) D[j][i] = r[j];
    }
    __syncthreads();
    const int row = kb + bw + blockIdx.x * blockDim.x + threadIdx.x;
    if (rows_here && row < F.nr) {
        T x[kNB];
#pragma unroll
        for (int k = 0; k < kNB; k++) x[k] = k < bw ? F.P[(i64)(kb + k) * F.nr + row] : T(0);
#pragma unroll
        for (int k = 0; k < kNB; k++) {
            if (k < bw) {
                T a = x[k];
#pragma unroll
                for (int m = 0; m < kNB; m++)
                    if (m < k) a -= x[m] * D[m][k];
                x[k] = a / D[k][k];
            }
        }
#pragma unroll
        for (int k = 0; k < kNB; k++)
            if (k < bw) F.P[(i64)(kb + k) * F.nr + row] = x[k];
    }
    // the last work-group of this (front, instance) stores the factored block
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        int* c = cnt + (i64)blockIdx.z * gridDim.y + blockIdx.y;
        const int done = atomicAdd(c, 1) + 1;
        last = done == nwg;
        if (last) atomicExch(c, 0);
    }
    __syncthreads();
    if (last) {
        __threadfence();
        for (int idx = threadIdx.x; idx < bw * bw; idx += blockDim.x) {
            const int j = idx / bw, i = idx - j * bw;
            if (j <= i) F.P[(i64)(kb + j) * F.nr + kb + i] = D[j][i];
        }
    }
}

template <typename T>
struct MfmaT;
template <>
struct MfmaT<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct MfmaT<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Update of a large front with its factored columns [ka, ka + R) (R <= 128,
// clipped to the front's width): C -= L21 L21^T over the target columns
// [c0, c1) (rows c0..nr-1, lower part), with c0 = ka + R. strip = 1: c1 =
// min(c0 + NB, w), the next panel only (left-looking inside a 128-column
// block); strip = 0: c1 = nr, the whole trailing matrix (once per block).
// Tile (ti, tj) of 64 x 64 from blockIdx.x = tj * nti + ti, ti >= tj; four
// wavefronts, each a 32 x 32 quarter as 2 x 2 MFMA blocks; the R columns are
// staged through LDS 32 at a time and accumulate in the MFMA registers.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_big_update(SymView S, const i32* __restrict__ fronts, int ka, int R,
                                                       int strip, int nti, T* __restrict__ L, T* __restrict__ CB,
                                                       const int* active) {
    __shared__ T Ai[kTile][kNB + 1];
    __shared__ T Aj[kTile][kNB + 1];
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const i32 s = fronts[blockIdx.y];
    const FrontRef<T> F = front_of<T>(S, s, b, L, CB);
    const int rf = min(R, F.w - ka);
    if (rf <= 0) return;
    const int c0 = ka + rf;
    const int c1 = strip ? min(c0 + kNB, F.w) : F.nr;
    if (c1 <= c0) return;
    const int tj = blockIdx.x / nti, ti = blockIdx.x - tj * nti;
    if (ti < tj) return;
    const int i0 = c0 + ti * kTile, j0 = c0 + tj * kTile;
    if (i0 >= F.nr || j0 >= c1) return;
    typedef typename MfmaT<T>::v4 v4;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int qi = (wv >> 1) * 32, qj = (wv & 1) * 32;
    v4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int c = 0; c < 2; c++) acc[a][c] = v4{T(0), T(0), T(0), T(0)};
    const int li = lane & 15, lk = lane >> 4;
    for (int kc = 0; kc < rf; kc += kNB) {
        const int bw = min(kNB, rf - kc);
        __syncthreads();   // previous chunk consumed
        for (int idx = threadIdx.x; idx < kTile * kNB; idx += blockDim.x) {
            const int k = idx / kTile, r = idx - k * kTile;
            const bool ok = k < bw;
            const i64 col = (i64)(ka + kc + k) * F.nr;
            Ai[r][k] = (ok && i0 + r < F.nr) ? F.P[col + i0 + r] : T(0);
            Aj[r][k] = (ok && j0 + r < F.nr) ? F.P[col + j0 + r] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < kNB; k4 += 4) {
            T av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; a++) av[a] = Ai[qi + 16 * a + li][k4 + lk];
#pragma unroll
            for (int c = 0; c < 2; c++) bv[c] = Aj[qj + 16 * c + li][k4 + lk];
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int c = 0; c < 2; c++) acc[a][c] = MfmaT<T>::mma(av[a], bv[c], acc[a][c]);
        }
    }
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int c = 0; c < 2; c++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int i = i0 + qi + 16 * a + MfmaT<T>::row(lane, r);
                const int j = j0 + qj + 16 * c + (lane & 15);
                if (i < F.nr && j < c1 && i >= j) F.at(i, j) -= acc[a][c][r];
            }
}

// The trailing update of a 128-column block (strip = 0 above) on 128 x 128
// tiles: eight wavefronts, each a 64 x 32 part as 4 x 2 MFMA blocks (an
// operand value read from LDS feeds two or four MFMAs), and the R columns
// stream through two LDS buffers of KC columns: the loads of chunk c + 1 are
// in flight while chunk c is multiplied, one barrier per chunk. Tile (ti,
// tj) from blockIdx.x = tj * nti + ti, ti >= tj; targets rows c0..nr-1,
// columns c0..nr-1 (lower part).
constexpr int kUpdTile = 128;
constexpr int kUpdThreads = 512;
template <typename T>
__host__ __device__ constexpr int upd2_kc() {
    // 16 columns per chunk in both precisions: 37 KiB (FP32) / 74 KiB (FP64)
    // of dynamic LDS for the two double buffers; 32 FP32 columns measured 1%
    // slower on a dense 20k factorization, 8 FP64 columns 2.4% slower
    return 16;
}
constexpr int kUpdPad = 16;            // row stride kUpdTile + 16: the four k rows of a read hit distinct banks
template <typename T>
__host__ __device__ constexpr int upd2_lds() {
    return 2 * 2 * upd2_kc<T>() * (kUpdTile + kUpdPad) * (int)sizeof(T);
}

template <typename T>
__global__ __launch_bounds__(kUpdThreads) void k_big_update2(SymView S, const i32* __restrict__ fronts, int ka,
                                                             int R, int nti, T* __restrict__ L, T* __restrict__ CB,
                                                             const int* active) {
    constexpr int KC = upd2_kc<T>();
    constexpr int LD = kUpdTile + kUpdPad;
    constexpr int NE = 2 * kUpdTile * KC / kUpdThreads;   // elements each thread stages per chunk (both operands)
    extern __shared__ double smem_u[];                    // upd2_lds<T>() bytes
    T (*buf)[2][KC][LD] = reinterpret_cast<T (*)[2][KC][LD]>(smem_u);   // [buffer][operand i / j][k][row]
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const i32 s = fronts[blockIdx.y];
    const FrontRef<T> F = front_of<T>(S, s, b, L, CB);
    const int rf = min(R, F.w - ka);
    if (rf <= 0) return;
    const int c0 = ka + rf;
    if (F.nr <= c0) return;
    const int tj = blockIdx.x / nti, ti = blockIdx.x - tj * nti;
    if (ti < tj) return;
    const int i0 = c0 + ti * kUpdTile, j0 = c0 + tj * kUpdTile;
    if (i0 >= F.nr) return;
    typedef typename MfmaT<T>::v4 v4;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int qi = (wv >> 2) * 64, qj = (wv & 3) * 32;
    const int li = lane & 15, lk = lane >> 4;
    v4 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 2; c++) acc[a][c] = v4{T(0), T(0), T(0), T(0)};
    // staging: element e of a thread is operand (e & 1) [i / j], flat index
    // f = (e >> 1) * kUpdThreads + threadIdx.x of the operand's KC x 128
    // block (k = f / 128, row = f % 128): consecutive threads read
    // consecutive rows of one column (coalesced)
    T st[NE];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int e = 0; e < NE; e++) {
            const int f = (e >> 1) * kUpdThreads + threadIdx.x;
            const int k = f / kUpdTile, r = f - k * kUpdTile;
            const int row = ((e & 1) ? j0 : i0) + r;
            const bool ok = kc + k < rf && row < F.nr;
            const i64 at = (i64)(ka + kc + min(k, rf - 1 - kc)) * F.nr + min(row, F.nr - 1);
            const T v = F.P[at];
            st[e] = ok ? v : T(0);
        }
    };
    auto stage = [&](int q) {
#pragma unroll
        for (int e = 0; e < NE; e++) {
            const int f = (e >> 1) * kUpdThreads + threadIdx.x;
            const int k = f / kUpdTile, r = f - k * kUpdTile;
            buf[q][e & 1][k][r] = st[e];
        }
    };
    fetch(0);
    stage(0);
    __syncthreads();
    int q = 0;
    for (int kc = 0; kc < rf; kc += KC) {
        const bool more = kc + KC < rf;
        if (more) fetch(kc + KC);
#pragma unroll
        for (int k4 = 0; k4 < KC; k4 += 4) {
            T av[4], bv[2];
#pragma unroll
            for (int a = 0; a < 4; a++) av[a] = buf[q][0][k4 + lk][qi + 16 * a + li];
#pragma unroll
            for (int c = 0; c < 2; c++) bv[c] = buf[q][1][k4 + lk][qj + 16 * c + li];
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int c = 0; c < 2; c++) acc[a][c] = MfmaT<T>::mma(av[a], bv[c], acc[a][c]);
        }
        if (more) stage(q ^ 1);
        __syncthreads();   // the other buffer is staged; this one is free again
        q ^= 1;
    }
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 2; c++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int i = i0 + qi + 16 * a + MfmaT<T>::row(lane, r);
                const int j = j0 + qj + 16 * c + li;
                if (i < F.nr && i >= j) F.at(i, j) -= acc[a][c][r];
            }
}

// the bw x bw diagonal tile whose first entry is panel entry (r0, r0) into
// D (leading dimension kTri), by a kBlock-thread work-group with every load
// in flight before the LDS stores (bw <= kTri)
template <typename T>
__device__ __forceinline__ void load_tile(T* D, const T* __restrict__ Lb, i64 nr, int r0, int bw) {
    constexpr int K = kTri * kTri / kBlock;
    T v[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int idx = min((int)threadIdx.x + k * kBlock, bw * bw - 1);
        const int jj = idx / bw, ii = idx - jj * bw;
        v[k] = Lb[(i64)(r0 + jj) * nr + r0 + ii];
    }
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int idx = (int)threadIdx.x + k * kBlock;
        if (idx < bw * bw) {
            const int jj = idx / bw, ii = idx - jj * bw;
            D[jj * kTri + ii] = v[k];
        }
    }
}

// ---------------------------------------------------------------------------
// supernodal triangular solves, one work-group per (supernode, instance) of a
// level. Forward (L y = b), multifrontal form: each supernode gathers its
// children's update vectors (the amount to subtract at their rows below),
// solves with its diagonal block and emits L21 y plus the pass-through part
// as its own update vector; no atomics, deterministic.
// Backward (L^T x = y), pull form: gather x at the rows below (ancestors,
// already final), subtract L21^T x, solve with L11^T.
// The diagonal block is staged in LDS in kTri x kTri tiles and solved by one
// wavefront with lane shuffles.
// ---------------------------------------------------------------------------
// GU: the working vector does not fit the LDS budget and lives in the solve
// vector (the supernode's columns) and in the supernode's update vector
// (rows below; forward only), with only the diagonal tile in LDS.
template <typename T, bool PUSH, bool GU>
__global__ __launch_bounds__(kBlock) void k_fwd(SymView S, const i32* __restrict__ list, const T* __restrict__ L,
                                                T* __restrict__ X, T* __restrict__ UV, const int* ids,
                                                const CGState* st) {
    extern __shared__ double smem_d[];
    T* D = reinterpret_cast<T*>(smem_d);
    T* u = D + kTri * kTri;
    const int b = inst_of(ids, blockIdx.y);
    const i32 s = list[blockIdx.x];
    if (st && st[(i64)b * S.G + (S.G > 1 ? S.sn_mem[s] : 0)].done) return;
    const i32 f = S.sn_first[s];
    const int w = S.sn_first[s + 1] - f;
    const int nr = (int)(S.sn_rowptr[s + 1] - S.sn_rowptr[s]);
    const T* Lb = L + (i64)b * S.Lsize + S.sn_lptr[s];
    T* x = X + (i64)b * S.n;
    T* uvb = UV + (i64)b * S.UVsize;
    T* ub = uvb + S.sn_uvptr[s];
    auto U = [&](int i) -> T& { return GU ? (i < w ? x[f + i] : ub[i - w]) : u[i]; };
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {
        if (!GU) u[i] = i < w ? x[f + i] : T(0);
        else if (i >= w) ub[i - w] = T(0);
    }
    __syncthreads();
    for (int q = S.child_ptr[s]; !PUSH && q < S.child_ptr[s + 1]; q++) {
        const i32 c = S.child_list[q];
        const int wc = S.sn_first[c + 1] - S.sn_first[c];
        const int ncc = (int)(S.sn_rowptr[c + 1] - S.sn_rowptr[c]) - wc;
        const i32* rel = S.relmap + S.sn_uvptr[c];
        const T* uc = uvb + S.sn_uvptr[c];
        for (int k = threadIdx.x; k < ncc; k += blockDim.x) U(rel[k]) += uc[k];
        __syncthreads();
    }
    for (int kb = 0; kb < w; kb += kTri) {
        const int bw = min(kTri, w - kb);
        load_tile(D, Lb, nr, kb, bw);
        __syncthreads();
        if (threadIdx.x < kWave) {
            const int lane = threadIdx.x;
            T val = lane < bw ? U(kb + lane) : T(0);
            for (int k = 0; k < bw; k++) {
                if (lane == k) val = val / D[k * kTri + k];
                const T yk = __shfl(val, k, kWave);
                if (lane > k && lane < bw) val -= D[k * kTri + lane] * yk;
            }
            if (lane < bw) U(kb + lane) = val;
        }
        __syncthreads();
        for (int i = kb + bw + threadIdx.x; i < nr; i += blockDim.x) {
            T sum = T(0);
            for (int k = 0; k < bw; k++) sum += Lb[(i64)(kb + k) * nr + i] * U(kb + k);
            U(i) -= sum;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {
        if (i < w) {
            if (!GU) x[f + i] = u[i];
        } else if (PUSH) {
            unsafeAtomicAdd(&x[S.sn_rows[S.sn_rowptr[s] + i]], U(i));
        } else if (!GU) {
            ub[i - w] = u[i];
        }
    }
}

template <typename T, bool GU>
__global__ __launch_bounds__(kBlock) void k_bwd(SymView S, const i32* __restrict__ list, const T* __restrict__ L,
                                                T* __restrict__ X, const int* ids, const CGState* st) {
    extern __shared__ double smem_d[];
    T* D = reinterpret_cast<T*>(smem_d);
    T* u = D + kTri * kTri;
    const int b = inst_of(ids, blockIdx.y);
    const i32 s = list[blockIdx.x];
    if (st && st[(i64)b * S.G + (S.G > 1 ? S.sn_mem[s] : 0)].done) return;
    const i32 f = S.sn_first[s];
    const int w = S.sn_first[s + 1] - f;
    const int nr = (int)(S.sn_rowptr[s + 1] - S.sn_rowptr[s]);
    const i32* rows = S.sn_rows + S.sn_rowptr[s];
    const T* Lb = L + (i64)b * S.Lsize + S.sn_lptr[s];
    T* x = X + (i64)b * S.n;
    // GU: columns in place in x, rows below read from x (ancestors, final)
    auto U = [&](int i) -> T& { return GU ? (i < w ? x[f + i] : x[rows[i]]) : u[i]; };
    if (!GU)
        for (int i = threadIdx.x; i < nr; i += blockDim.x) u[i] = i < w ? x[f + i] : x[rows[i]];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int nblk = (w + kTri - 1) / kTri;
    for (int kbi = nblk - 1; kbi >= 0; kbi--) {
        const int kb = kbi * kTri;
        const int bw = min(kTri, w - kb);
        for (int jj = wid; jj < bw; jj += nw) {
            const int j = kb + jj;
            T sum = T(0);
            for (int i = kb + bw + lane; i < nr; i += kWave) sum += Lb[(i64)j * nr + i] * U(i);
            sum = wave_sum(sum);
            if (lane == 0) U(j) -= sum;
        }
        load_tile(D, Lb, nr, kb, bw);
        __syncthreads();
        if (threadIdx.x < kWave) {
            T val = lane < bw ? U(kb + lane) : T(0);
            for (int k = bw - 1; k >= 0; k--) {
                if (lane == k) val = val / D[k * kTri + k];
                const T xk = __shfl(val, k, kWave);
                if (lane < k) val -= D[lane * kTri + k] * xk;
            }
            if (lane < bw) U(kb + lane) = val;
        }
        __syncthreads();
    }
    if (!GU)
        for (int i = threadIdx.x; i < w; i += blockDim.x) x[f + i] = u[i];
}

// ---------------------------------------------------------------------------
// Wide supernodes (more than 1024 rows or columns): blocked triangular solves
// spread over many work-groups, right-looking forward solve with FP atomics
// for the rows below the supernode. The w columns of the panel are cut into
// diagonal blocks of kWsB columns.
// Forward, launch q: every work-group but the first applies block q-1's
// solution (final since launch q-1) to kWsR rows below that block; the first
// work-group owns block q's rows, applies block q-1 to them and then solves
// block q with its diagonal triangle (look-ahead: one launch per block, the
// rows of block q are final once block q-1 is applied).
// Backward: one launch subtracts the rows below the supernode (ancestors'
// x, final) from every column; then launch q (last block first) applies
// block q+1's solution to kWsR columns left of block q per work-group, and
// the first work-group, owning block q's columns, applies it to them and
// solves block q with the transposed triangle.
// Grid: x = work-group of the supernode (0 = owner), y = supernode of the
// level's list, z = instance list index. All work of a supernode sits in
// its panel (column-major, nr x w, leading dimension nr).
// ---------------------------------------------------------------------------
constexpr int kWsB = 256;   // columns per diagonal block (= threads of the owner work-group)
constexpr int kWsR = 64;    // rows (forward) / columns (backward) per update work-group

static_assert(kWsB == kBlock, "the owner work-group holds one block row per thread");

// sum_{j < n} col[j * ld] * v[j], sixteen independent loads in flight
template <typename T>
__device__ __forceinline__ T strided_dot(const T* __restrict__ col, i64 ld, const T* v, int n) {
    T sum = T(0);
    int j = 0;
    for (; j + 16 <= n; j += 16) {
        T l[16];
#pragma unroll
        for (int u = 0; u < 16; u++) l[u] = col[(i64)(j + u) * ld];
#pragma unroll
        for (int u = 0; u < 16; u++) sum += l[u] * v[j + u];
    }
    for (; j < n; j++) sum += col[(i64)j * ld] * v[j];
    return sum;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_ws_fwd(SymView S, const TriDesc* __restrict__ desc, int q,
                                                   const T* __restrict__ L, T* __restrict__ X, const int* ids,
                                                   const CGState* st) {
    __shared__ T ys[kWsB];                       // block q-1's solution
    __shared__ T part[kBlock / kWave][kWave];    // partial row sums of the waves
    __shared__ T D[kTri * kTri];                 // owner: diagonal tile
    __shared__ T u[kWsB];                        // owner: the block's right-hand side, then solution
    const TriDesc d = desc[blockIdx.y];
    const int b = inst_of(ids, blockIdx.z);
    if (st && st[(i64)b * S.G + d.mem].done) return;
    const int w = d.w, nr = d.nr;
    const int a = (q - 1) * kWsB;                // applied block [a, e)
    const bool apply = q > 0 && a < w;
    const int e = apply ? min(a + kWsB, w) : a;
    const int qb = q * kWsB;
    const int s0 = min(qb + kWsB, w);            // rows of the update work-groups start here
    const bool owner = blockIdx.x == 0;
    int r_lo, r_hi;
    if (owner) {
        if (qb >= w) return;
        r_lo = qb;
        r_hi = s0;
    } else {
        if (!apply) return;
        r_lo = s0 + (int)(blockIdx.x - 1) * kWsR;
        if (r_lo >= nr) return;
        r_hi = min(r_lo + kWsR, nr);
    }
    const T* Lb = L + (i64)b * S.Lsize + d.lptr;
    T* x = X + (i64)b * S.n;
    const int na = e - a;
    for (int j = threadIdx.x; apply && j < na; j += blockDim.x) ys[j] = x[d.f + a + j];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (!owner) {
        // kWsR = 64 rows, the waves split the applied block's columns
        const int r = r_lo + lane;
        const int per = (na + (kBlock / kWave) - 1) / (kBlock / kWave);
        const int j0 = min(wid * per, na), j1 = min(j0 + per, na);
        T sum = T(0);
        if (r < r_hi) sum = strided_dot(Lb + (i64)(a + j0) * nr + r, nr, ys + j0, j1 - j0);
        part[wid][lane] = sum;
        __syncthreads();
        if (wid == 0 && r < r_hi) {
            T t = part[0][lane];
#pragma unroll
            for (int k = 1; k < kBlock / kWave; k++) t += part[k][lane];
            if (r < w) x[d.f + r] -= t;
            else unsafeAtomicAdd(&x[S.sn_rows[d.rp + r]], -t);
        }
        return;
    }
    // owner: rows [qb, s0) of block q, one per thread
    const int bw = s0 - qb;
    const int t = threadIdx.x;
    T val = T(0);
    if (t < bw) {
        val = x[d.f + qb + t];
        if (apply) val -= strided_dot(Lb + (i64)a * nr + qb + t, nr, ys, na);
    }
    u[t] = val;
    __syncthreads();
    for (int kb = 0; kb < bw; kb += kTri) {
        const int tw = min(kTri, bw - kb);
        load_tile(D, Lb, nr, qb + kb, tw);
        __syncthreads();
        if (wid == 0) {
            T v = lane < tw ? u[kb + lane] : T(0);
            for (int k = 0; k < tw; k++) {
                if (lane == k) v = v / D[k * kTri + k];
                const T yk = __shfl(v, k, kWave);
                if (lane > k && lane < tw) v -= D[k * kTri + lane] * yk;
            }
            if (lane < tw) u[kb + lane] = v;
        }
        __syncthreads();
        if (t >= kb + tw && t < bw) u[t] -= strided_dot(Lb + (i64)(qb + kb) * nr + qb + t, nr, u + kb, tw);
        __syncthreads();
    }
    if (t < bw) x[d.f + qb + t] = u[t];
}

// Backward, rows below the supernode: x_j -= sum_{r >= w} L(r, j) x(row r)
// for the kWsR columns of this work-group (one wave per column at a time).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ws_bwd_below(SymView S, const TriDesc* __restrict__ desc,
                                                         const T* __restrict__ L, T* __restrict__ X,
                                                         const int* ids, const CGState* st) {
    const TriDesc d = desc[blockIdx.y];
    const int b = inst_of(ids, blockIdx.z);
    if (st && st[(i64)b * S.G + d.mem].done) return;
    const int w = d.w, nr = d.nr;
    const int c0 = (int)blockIdx.x * kWsR;
    if (c0 >= w || nr == w) return;
    const T* Lb = L + (i64)b * S.Lsize + d.lptr;
    T* x = X + (i64)b * S.n;
    const i32* rows = S.sn_rows + d.rp;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    // eight row chunks of the wave in flight: their row indices, then the
    // panel entries and the gathered x together
    for (int j = c0 + wid; j < min(c0 + kWsR, w); j += kBlock / kWave) {
        const T* col = Lb + (i64)j * nr;
        T sum = T(0);
        for (int r0 = w + lane; r0 < nr; r0 += 8 * kWave) {
            i32 ri[8];
#pragma unroll
            for (int k = 0; k < 8; k++) ri[k] = rows[min(r0 + k * kWave, nr - 1)];
            T lv[8], xv[8];
#pragma unroll
            for (int k = 0; k < 8; k++) {
                lv[k] = col[min(r0 + k * kWave, nr - 1)];
                xv[k] = x[ri[k]];
            }
#pragma unroll
            for (int k = 0; k < 8; k++)
                if (r0 + k * kWave < nr) sum += lv[k] * xv[k];
        }
        sum = wave_sum(sum);
        if (lane == 0) x[d.f + j] -= sum;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_ws_bwd(SymView S, const TriDesc* __restrict__ desc, int q,
                                                   const T* __restrict__ L, T* __restrict__ X, const int* ids,
                                                   const CGState* st) {
    __shared__ T xs[kWsB];                       // block q+1's solution
    __shared__ T D[kTri * kTri];                 // owner: diagonal tile
    __shared__ T u[kWsB];                        // owner: the block's right-hand side, then solution
    const TriDesc d = desc[blockIdx.y];
    const int b = inst_of(ids, blockIdx.z);
    if (st && st[(i64)b * S.G + d.mem].done) return;
    const int w = d.w, nr = d.nr;
    const int qb = q * kWsB;
    if (qb >= w) return;                         // this supernode has no block q
    const int a = qb + kWsB;                     // applied block [a, e)
    const bool apply = a < w;
    const int e = apply ? min(a + kWsB, w) : a;
    const bool owner = blockIdx.x == 0;
    int c_lo, c_hi;
    if (owner) {
        c_lo = qb;
        c_hi = min(qb + kWsB, w);
    } else {
        if (!apply) return;
        c_lo = (int)(blockIdx.x - 1) * kWsR;
        if (c_lo >= qb) return;
        c_hi = min(c_lo + kWsR, qb);
    }
    const T* Lb = L + (i64)b * S.Lsize + d.lptr;
    T* x = X + (i64)b * S.n;
    const int na = e - a;
    for (int j = threadIdx.x; apply && j < na; j += blockDim.x) xs[j] = x[d.f + a + j];
    if (owner)
        for (int j = threadIdx.x; j < c_hi - c_lo; j += blockDim.x) u[j] = x[d.f + c_lo + j];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    // columns j in [c_lo, c_hi): x_j -= sum_{i in [a, e)} L(i, j) x_i: the
    // applied rows of a column are a contiguous run, loaded 16 at a time.
    // The owner takes one thread per column (kWsB = threads); an update
    // work-group (kWsR = 64 columns) one lane per column with the applied
    // rows split in four quarters over the waves, the four partial sums
    // added in LDS
    if (owner) {
        const int j = c_lo + (int)threadIdx.x;
        if (apply && j < c_hi) {
            const T* col = Lb + (i64)j * nr + a;
            T sum = T(0);
            for (int i0 = 0; i0 < na; i0 += 16) {
                T l[16];
#pragma unroll
                for (int k = 0; k < 16; k++) l[k] = col[min(i0 + k, na - 1)];
#pragma unroll
                for (int k = 0; k < 16; k++)
                    if (i0 + k < na) sum += l[k] * xs[i0 + k];
            }
            u[j - c_lo] -= sum;
        }
    } else {
        __shared__ T part[kBlock / kWave][kWave];
        static_assert(kWsR == kWave, "an update work-group holds one column per lane");
        const int j = c_lo + lane;
        const int per = (na + (kBlock / kWave) - 1) / (kBlock / kWave);
        const int i_lo = min(wid * per, na), i_hi = min(i_lo + per, na);
        T sum = T(0);
        if (j < c_hi) {
            const T* col = Lb + (i64)j * nr + a;
            for (int i0 = i_lo; i0 < i_hi; i0 += 16) {
                T l[16];
#pragma unroll
                for (int k = 0; k < 16; k++) l[k] = col[min(i0 + k, i_hi - 1)];
#pragma unroll
                for (int k = 0; k < 16; k++)
                    if (i0 + k < i_hi) sum += l[k] * xs[i0 + k];
            }
        }
        part[wid][lane] = sum;
        __syncthreads();
        if (wid == 0 && j < c_hi) {
            T t = part[0][lane];
#pragma unroll
            for (int k = 1; k < kBlock / kWave; k++) t += part[k][lane];
            x[d.f + j] -= t;
        }
        return;
    }
    __syncthreads();
    // owner: transposed solve of block q, last 64-column tile first
    const int bw = c_hi - c_lo;
    const int ntile = (bw + kTri - 1) / kTri;
    for (int ti = ntile - 1; ti >= 0; ti--) {
        const int kb = ti * kTri;
        const int tw = min(kTri, bw - kb);
        load_tile(D, Lb, nr, qb + kb, tw);
        __syncthreads();
        if (wid == 0) {
            T v = lane < tw ? u[kb + lane] : T(0);
            for (int k = tw - 1; k >= 0; k--) {
                if (lane == k) v = v / D[k * kTri + k];
                const T xk = __shfl(v, k, kWave);
                if (lane < k) v -= D[lane * kTri + k] * xk;
            }
            if (lane < tw) u[kb + lane] = v;
        }
        __syncthreads();
        // earlier columns of the block: u_j -= sum_{i in tile} L(qb+kb+i, qb+j)
        // u_{kb+i}, one thread per column j < kb (kb < kWsB = threads): the
        // tile's rows of a column are contiguous, loaded 16 at a time
        if ((int)threadIdx.x < kb) {
            const T* col = Lb + (i64)(qb + threadIdx.x) * nr + qb + kb;
            T sum = T(0);
            for (int i0 = 0; i0 < tw; i0 += 16) {
                T l[16];
#pragma unroll
                for (int k = 0; k < 16; k++) l[k] = col[min(i0 + k, tw - 1)];
#pragma unroll
                for (int k = 0; k < 16; k++)
                    if (i0 + k < tw) sum += l[k] * u[kb + i0 + k];
            }
            u[threadIdx.x] -= sum;
        }
        __syncthreads();
    }
    for (int j = threadIdx.x; j < bw; j += blockDim.x) x[d.f + qb + j] = u[j];
}

// ---------------------------------------------------------------------------
// wavefront triangular solves: a wavefront is split into 64/SEG segments of
// SEG lanes; each segment solves one (supernode, instance) task, all
// segments of a wavefront the same supernode for consecutive instances (the
// task space of a supernode is padded to a multiple of 64/SEG, so control
// flow is uniform). Rows across the lanes of a segment (R rows per lane,
// nr <= SEG*R), panel columns prefetched kChunk at a time into registers
// (coalesced column loads), the pivot broadcast by a segment shuffle. No LDS
// and no work-group barriers.
// Forward: v = [x(cols); 0] + children's update vectors (pulled through the
// per-row gather list); for each column j: y_j = v_j / L_jj, v_i -= L_ij y_j;
// rows below the block leave as this supernode's update vector.
// Backward: v = [y(cols); x(rows below)]; for j = w-1..0:
// x_j = (v_j - sum_{i>j} L_ij x_i) / L_jj with a butterfly segment sum.
// ---------------------------------------------------------------------------
// panel columns fetched per memory round trip: 16 for the 64-lane class with
// one row per lane, 8 otherwise, but for sixteen rows per lane 4 (FP32) or 2
// (FP64): more columns of that height do not fit the 256 vector registers
// next to the rows, and the compiler then parks each loaded value in the
// accumulation registers and waits for it, one load at a time
template <typename T, int SEG, int R>
__host__ __device__ constexpr int chunk_cols() {
    return (SEG == 64 && R == 1) ? 16 : R >= 16 ? (sizeof(T) == 8 ? 2 : 4) : 8;
}

// Lane permutations within rows of 16 lanes through DPP (a VALU operand
// modifier, no LDS round trip): quad_perm [1,0,3,2], quad_perm [2,3,0,1],
// row_half_mirror (lane i <-> 7-i within 8), row_mirror (i <-> 15-i).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the SEG lanes of a segment, the same value in every lane of it:
// butterfly over lane pairs, the steps within 16 lanes by DPP, the 16- and
// 32-lane steps by lane permutes. Each step adds equal partial sums, so all
// lanes end with bitwise equal results.
template <typename T, int SEG>
__device__ __forceinline__ T seg_allsum(T v) {
    v += dpp_mov<0xB1>(v);                          // pairs
    v += dpp_mov<0x4E>(v);                          // quads
    if (SEG >= 8) v += dpp_mov<0x141>(v);           // 8 lanes
    if (SEG >= 16) v += dpp_mov<0x140>(v);          // 16 lanes
    if (SEG >= 32) v += __shfl_xor(v, 16, SEG);
    if (SEG >= 64) v += __shfl_xor(v, 32, SEG);
    return v;
}

// Value of lane jl of the segment in every lane of it. A 64-lane segment is
// the whole wavefront, whose column loop runs in lockstep, so jl is uniform
// and v_readlane serves. When every segment of the wavefront is at the same
// column (U: the per-level kernels, whose segments share a supernode), lane
// jl of each segment is read with v_readlane and each lane keeps its own
// segment's value (a readlane is several times cheaper than a lane permute
// through LDS); otherwise (segments of a tree-kernel wavefront may sit at
// different columns) a lane permute.
template <typename T, int SEG, bool U>
__device__ __forceinline__ T seg_bcast(T v, int jl) {
    if (SEG == kWave) return lane_read(v, jl);
    if (U) {
        const int sg = (int)(threadIdx.x & (kWave - 1)) / SEG;
        T r = lane_read(v, jl);
#pragma unroll
        for (int k = 1; k < kWave / SEG; k++) {
            const T a = lane_read(v, jl + k * SEG);
            r = sg == k ? a : r;
        }
        return r;
    }
    return __shfl(v, jl, SEG);
}

// PUSH = false: children's update vectors are pulled through the gather list
// (deterministic). PUSH = true: the rows below the diagonal block are added
// straight into the ancestors' right-hand-side entries with FP atomics
// (right-looking; order of the additions not fixed).
// Load panel columns [j0, j0 + CH) of the rows this lane holds (strictly
// below the diagonal, zero elsewhere). Every lane loads from an address
// clamped into the panel and selects afterwards: no branch per element.
// PK: Lb is the supernode's packed solve copy (strictly lower entries only,
// column jc starting at jc (nr - 1) - jc (jc - 1) / 2, one padding entry at
// Lb[-1]), else its panel. With jc and the row clamped, the packed entry
// index of (row, jc) is jc (2 nr - 3 - jc) / 2 - 1 + row (an exact halving),
// which stays in [-1, entries): no further clamp.
template <typename T, int SEG, int R, int CH, bool PK, typename DT>
__device__ __forceinline__ void load_cols(T (&lc)[CH][R], const T* __restrict__ Lb, const DT& d, int j0, int sl) {
#pragma unroll
    for (int jj = 0; jj < CH; jj++) {
        const int j = j0 + jj;
        const int jc = min(max(j, 0), d.w - 1);
        const int cst = PK ? ((jc * (2 * d.nr - 3 - jc)) >> 1) - 1 : jc * d.nr;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int row = sl + SEG * r;
            const T val = Lb[cst + min(row, d.nr - 1)];
            lc[jj][r] = (j >= 0 && j < d.w && row > j && row < d.nr) ? val : T(0);
        }
    }
}

// One (supernode d, instance b) task on the SEG lanes of this thread's
// segment. Loads depend on the descriptor and b only (b is a valid instance
// even for an invalid task), so they are issued without waiting for the
// validity test, and the first chunk of panel columns goes out together
// with the right-hand-side entries; valid only gates the stores.
// Forward substitution over the panel columns on the rows this lane holds:
// v enters as the right-hand side (rows of the diagonal block) or zero
// (rows below) and leaves as the solution or the update for the rows below.
// lc holds the first chunk of columns on entry.
template <typename T, int SEG, int R, int CH, bool U, bool PK, typename DT>
__device__ __forceinline__ void fwd_cols(T (&lc)[CH][R], T (&v)[R], const T (&di)[R], const T* __restrict__ Lb,
                                         const DT& d, int sl) {
    for (int j0 = 0; j0 < d.w; j0 += CH) {
        if (j0 > 0) load_cols<T, SEG, R, CH, PK>(lc, Lb, d, j0, sl);
#pragma unroll
        for (int jj = 0; jj < CH; jj++) {
            const int j = j0 + jj;
            if (j < d.w) {
                const int jl = j & (SEG - 1), jr = j / SEG;
                T vs = v[0], es = di[0];
#pragma unroll
                for (int r = 1; r < R; r++)
                    if (r == jr) { vs = v[r]; es = di[r]; }
                const T yj = seg_bcast<T, SEG, U>(vs * es, jl);      // y_j = v_j / L_jj, formed in lane jl
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const int row = sl + SEG * r;
                    if (row == j) v[r] = yj;
                    else v[r] -= lc[jj][r] * yj;      // zero below-diagonal mask for rows <= j
                }
            }
        }
    }
}

// Backward substitution, columns from the last one down: v enters as the
// right-hand side on the diagonal rows and the known solution on the rows
// below, and leaves with the solution on the diagonal rows. lc holds the
// chunk [w - CH, w) on entry.
template <typename T, int SEG, int R, int CH, bool U, bool PK, typename DT>
__device__ __forceinline__ void bwd_cols(T (&lc)[CH][R], T (&v)[R], const T (&di)[R], const T* __restrict__ Lb,
                                         const DT& d, int sl) {
    for (int jhi = d.w; jhi > 0; jhi -= CH) {
        const int j0 = jhi - CH;
        if (jhi < d.w) load_cols<T, SEG, R, CH, PK>(lc, Lb, d, j0, sl);
#pragma unroll
        for (int jj = CH - 1; jj >= 0; jj--) {
            const int j = j0 + jj;
            if (j >= 0) {
                T part = T(0);
#pragma unroll
                for (int r = 0; r < R; r++) part += lc[jj][r] * v[r];   // rows <= j are masked to zero
                part = seg_allsum<T, SEG>(part);
                const int jl = j & (SEG - 1), jr = j / SEG;
                T vs = v[0], es = di[0];
#pragma unroll
                for (int r = 1; r < R; r++)
                    if (r == jr) { vs = v[r]; es = di[r]; }
                const T xj = seg_bcast<T, SEG, U>((vs - part) * es, jl);   // formed in lane jl
#pragma unroll
                for (int r = 0; r < R; r++)
                    if (sl + SEG * r == j) v[r] = xj;
            }
        }
    }
}

// Lp: the packed solve copy (LPsize entries per instance)
template <typename T, int SEG, int R, bool PUSH, bool U>
__device__ __forceinline__ void fwd_body(const SymView& S, const TriDesc& d, int b, bool valid,
                                         const T* __restrict__ Lp, const T* __restrict__ Dinv, T* __restrict__ X,
                                         T* __restrict__ UV) {
    constexpr int CH = chunk_cols<T, SEG, R>();
    const int sl = threadIdx.x & (SEG - 1);
    const T* Lb = Lp + (i64)b * S.LPsize + d.pptr;
    const T* dinv = Dinv + (i64)b * S.n + d.f;
    T* x = X + (i64)b * S.n;
    T* uvb = UV + (i64)b * S.UVsize;
    T lc[CH][R];
    load_cols<T, SEG, R, CH, true>(lc, Lb, d, 0, sl);
    T v[R], di[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int row = sl + SEG * r;
        T a = T(0), e = T(0);
        if (row < d.w) {
            a = x[d.f + row];
            e = dinv[row];
        }
        if (!PUSH && row < d.nr && d.nchild) {
            const int g0 = S.ga_row[2 * (d.rp + row)], gn = S.ga_row[2 * (d.rp + row) + 1];
            for (int g = g0; g < g0 + gn; g++) a += uvb[S.ga_idx[g]];
        }
        v[r] = a;
        di[r] = e;
    }
    fwd_cols<T, SEG, R, CH, U, true>(lc, v, di, Lb, d, sl);
    if (!valid) return;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int row = sl + SEG * r;
        if (row < d.w) x[d.f + row] = v[r];
        else if (row < d.nr) {
            if (PUSH) unsafeAtomicAdd(&x[S.sn_rows[d.rp + row]], v[r]);
            else uvb[d.uvptr + row - d.w] = v[r];
        }
    }
}

template <typename T, int SEG, int R, bool U>
__device__ __forceinline__ void bwd_body(const SymView& S, const TriDesc& d, int b, bool valid,
                                         const T* __restrict__ Lp, const T* __restrict__ Dinv, T* __restrict__ X) {
    constexpr int CH = chunk_cols<T, SEG, R>();
    const int sl = threadIdx.x & (SEG - 1);
    const T* Lb = Lp + (i64)b * S.LPsize + d.pptr;
    const T* dinv = Dinv + (i64)b * S.n + d.f;
    T* x = X + (i64)b * S.n;
    // columns from the last one down in chunks [jhi - CH, jhi); the first
    // chunk goes out with the vector loads
    T lc[CH][R];
    load_cols<T, SEG, R, CH, true>(lc, Lb, d, d.w - CH, sl);
    T v[R], di[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int row = sl + SEG * r;
        T a = T(0), e = T(0);
        if (row < d.nr) a = row < d.w ? x[d.f + row] : x[S.sn_rows[d.rp + row]];
        if (row < d.w) e = dinv[row];
        v[r] = a;
        di[r] = e;
    }
    bwd_cols<T, SEG, R, CH, U, true>(lc, v, di, Lb, d, sl);
    if (!valid) return;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int row = sl + SEG * r;
        if (row < d.w) x[d.f + row] = v[r];
    }
}


// Index of this thread's wavefront in the work-group, as a wave-uniform
// value (the compiler does not infer that threadIdx.x / 64 is uniform): the
// task lookup below then runs on the scalar unit and the supernode's
// descriptor arrives through scalar loads.
__device__ __forceinline__ int wave_in_block() { return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); }

// Per-level mapping: all segments of a wavefront take the same supernode for
// consecutive entries of the instance list (the task space of a supernode is
// padded to a multiple of 64/SEG, so control flow is wave-uniform).
template <typename T, int SEG, int R, bool PUSH>
__device__ __forceinline__ void fwd_task(const SymView& S, const TriDesc* __restrict__ desc, int count, int npad,
                                         i64 wave, const T* __restrict__ Lp, const T* __restrict__ Dinv,
                                         T* __restrict__ X, T* __restrict__ UV, const int* ids, int nids,
                                         const CGState* st) {
    constexpr int G = kWave / SEG;
    const int seg = (threadIdx.x & (kWave - 1)) / SEG;
    const i64 t0 = wave * G;
    const int q = (int)(t0 / npad);
    if (q >= count) return;
    const int k = (int)(t0 - (i64)q * npad) + seg;
    bool valid = k < nids;
    const int b = valid ? inst_of(ids, k) : 0;
    const TriDesc d = desc[q];
    if (valid && st && st[(i64)b * S.G + d.mem].done) valid = false;
    fwd_body<T, SEG, R, PUSH, true>(S, d, b, valid, Lp, Dinv, X, UV);
}

template <typename T, int SEG, int R>
__device__ __forceinline__ void bwd_task(const SymView& S, const TriDesc* __restrict__ desc, int count, int npad,
                                         i64 wave, const T* __restrict__ Lp, const T* __restrict__ Dinv,
                                         T* __restrict__ X, const int* ids, int nids, const CGState* st) {
    constexpr int G = kWave / SEG;
    const int seg = (threadIdx.x & (kWave - 1)) / SEG;
    const i64 t0 = wave * G;
    const int q = (int)(t0 / npad);
    if (q >= count) return;
    const int k = (int)(t0 - (i64)q * npad) + seg;
    bool valid = k < nids;
    const int b = valid ? inst_of(ids, k) : 0;
    const TriDesc d = desc[q];
    if (valid && st && st[(i64)b * S.G + d.mem].done) valid = false;
    bwd_body<T, SEG, R, true>(S, d, b, valid, Lp, Dinv, X);
}

// ---------------------------------------------------------------------------
// Tree traversal: one work-group per instance walks a range of levels of the
// supernodal tree (forward: up; backward: down) with a work-group barrier
// between levels instead of a kernel boundary, so the instances progress
// independently and a level costs no launch. Meant for the thin upper
// levels, where a per-level launch is latency-bound; the wide lower levels
// need the whole chip per level. Within a
// level every segment of SEG lanes takes its own supernode of the class
// (segments of one wavefront may hold different supernodes; all shuffles
// stay inside a segment). seg[2 * (l * kTriClasses + c)] = (offset, count)
// of the supernodes of level l, class c in desc. Classes 0..kTreeClasses-1
// only; the host routes other levels to the per-level kernels.
// ---------------------------------------------------------------------------
constexpr int kTreeClasses = 5;


template <typename T, int SEG, int R, bool PUSH>
__device__ __forceinline__ void fwd_tree_class(const SymView& S, const TriDesc* __restrict__ desc, int cnt, int b,
                                               const T* __restrict__ Lp, const T* __restrict__ Dinv,
                                               T* __restrict__ X, T* __restrict__ UV, const CGState* st) {
    constexpr int G = kWave / SEG;
    const int wv = wave_in_block(), nw = blockDim.x / kWave;
    const int seg = (threadIdx.x & (kWave - 1)) / SEG;
    for (int base = wv * G; base < cnt; base += nw * G) {
        const int q = base + seg;
        bool valid = q < cnt;
        const TriDesc d = desc[valid ? q : cnt - 1];
        if (valid && st && st[(i64)b * S.G + d.mem].done) valid = false;
        fwd_body<T, SEG, R, PUSH, false>(S, d, b, valid, Lp, Dinv, X, UV);
    }
}

template <typename T, int SEG, int R>
__device__ __forceinline__ void bwd_tree_class(const SymView& S, const TriDesc* __restrict__ desc, int cnt, int b,
                                               const T* __restrict__ Lp, const T* __restrict__ Dinv,
                                               T* __restrict__ X, const CGState* st) {
    constexpr int G = kWave / SEG;
    const int wv = wave_in_block(), nw = blockDim.x / kWave;
    const int seg = (threadIdx.x & (kWave - 1)) / SEG;
    for (int base = wv * G; base < cnt; base += nw * G) {
        const int q = base + seg;
        bool valid = q < cnt;
        const TriDesc d = desc[valid ? q : cnt - 1];
        if (valid && st && st[(i64)b * S.G + d.mem].done) valid = false;
        bwd_body<T, SEG, R, false>(S, d, b, valid, Lp, Dinv, X);
    }
}

// forward over levels [l0, l1), then backward from l1-1 down to l0 (the
// levels above l1 are empty: the range ends at the root), one work-group
// per listed instance
template <typename T, bool PUSH, int NT>
__global__ __launch_bounds__(NT) void k_tri_tree(SymView S, const TriDesc* __restrict__ desc,
                                                 const i32* __restrict__ seg, int l0, int l1, const T* __restrict__ Lp,
                                                 const T* __restrict__ Dinv, T* __restrict__ X, T* __restrict__ UV,
                                                 const int* ids, const CGState* st) {
    const int b = inst_of(ids, blockIdx.x);
    for (int l = l0; l < l1; l++) {
        const i32* sg = seg + 2 * (l * kTriClasses);
        if (sg[1]) fwd_tree_class<T, 16, 1, PUSH>(S, desc + sg[0], sg[1], b, Lp, Dinv, X, UV, st);
        if (sg[3]) fwd_tree_class<T, 32, 1, PUSH>(S, desc + sg[2], sg[3], b, Lp, Dinv, X, UV, st);
        if (sg[5]) fwd_tree_class<T, 64, 1, PUSH>(S, desc + sg[4], sg[5], b, Lp, Dinv, X, UV, st);
        if (sg[7]) fwd_tree_class<T, 64, 2, PUSH>(S, desc + sg[6], sg[7], b, Lp, Dinv, X, UV, st);
        if (sg[9]) fwd_tree_class<T, 64, 4, PUSH>(S, desc + sg[8], sg[9], b, Lp, Dinv, X, UV, st);
        __syncthreads();
    }
    for (int l = l1 - 1; l >= l0; l--) {
        const i32* sg = seg + 2 * (l * kTriClasses);
        if (sg[1]) bwd_tree_class<T, 16, 1>(S, desc + sg[0], sg[1], b, Lp, Dinv, X, st);
        if (sg[3]) bwd_tree_class<T, 32, 1>(S, desc + sg[2], sg[3], b, Lp, Dinv, X, st);
        if (sg[5]) bwd_tree_class<T, 64, 1>(S, desc + sg[4], sg[5], b, Lp, Dinv, X, st);
        if (sg[7]) bwd_tree_class<T, 64, 2>(S, desc + sg[6], sg[7], b, Lp, Dinv, X, st);
        if (sg[9]) bwd_tree_class<T, 64, 4>(S, desc + sg[8], sg[9], b, Lp, Dinv, X, st);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Tree traversal with the whole working set of the top levels in LDS.
//
// Every row of a supernode in the top levels is a column of the supernode or
// of one of its ancestors, all of them in the top levels too, so the entries
// of x (and of the reciprocal diagonal) those levels touch form a closed set:
// they are read into LDS once, the forward updates go to LDS with LDS
// atomics, the backward solve reads them there, and x is written back once.
// The panels of a level are one contiguous range of L storage (panels are
// stored level by level); the work-group stages the next level's range in
// registers while it solves the current level from LDS, so a level costs no
// dependent global round trip.
//
// One wavefront per supernode. Forward (lane = row): the columns are scaled
// by the reciprocal diagonal when read, so that a column step is a lane
// broadcast of the running right-hand side entry and one FMA per row held.
// Backward (lane = column of the diagonal block): the rows below the
// diagonal block (ancestors, already solved) are first folded in by per-lane
// dot products, then the triangle is swept from the last column down with
// the same broadcast-and-FMA step; no cross-lane reductions.
// ---------------------------------------------------------------------------

// byte offsets of the LDS areas of k_tri_tree2 (the staged panels keep the
// layout of L storage)
struct Tree2Lds {
    int xs, dv, desc, rs, lvd, lvp, done, pan, total;
};
__host__ __device__ inline int al16(int v) { return (v + 15) & ~15; }
__host__ __device__ inline Tree2Lds tree2_layout(int nt, int esz, int nd, int nrs, int nlev, int G, int pmax) {
    Tree2Lds o;
    o.xs = 0;
    o.dv = al16(nt * esz);
    o.desc = al16(o.dv + nt * esz);
    o.rs = al16(o.desc + nd * (int)sizeof(TreeDesc));
    o.lvd = al16(o.rs + nrs * 4);
    o.lvp = al16(o.lvd + (nlev + 1) * 4);
    o.done = al16(o.lvp + (nlev + 1) * 8);
    o.pan = al16(o.done + G * 4);
    o.total = al16(o.pan + pmax * esz);
    return o;
}

// panel staging registers per thread (a level of at most NT * PR entries)
template <typename T>
__host__ __device__ constexpr int tree2_pr() {
    return 32;
}

// columns per chunk of the column loops (register budget of 64 words)
template <typename T, int R>
__host__ __device__ constexpr int tree2_chunk() {
    return (64 / (R * (int)(sizeof(T) / 4))) < 32 ? 64 / (R * (int)(sizeof(T) / 4)) : 32;
}

// staging of a level's ne panel entries by nl threads (thread t holds
// entries t, t + nl, ...)
template <typename T, int PR>
__device__ __forceinline__ void tree2_load(T (&pr)[PR], const T* __restrict__ src, int ne, int t, int nl) {
#pragma unroll
    for (int k = 0; k < PR; k++)
        if (k * nl < ne) pr[k] = src[min(k * nl + t, ne - 1)];
}

template <typename T, int PR>
__device__ __forceinline__ void tree2_store(const T (&pr)[PR], T* P, int ne, int t, int nl) {
#pragma unroll
    for (int k = 0; k < PR; k++) {
        const int e = k * nl + t;
        if (k * nl < ne && e < ne) P[e] = pr[k];
    }
}

// The staged kernel solves with the unit lower triangular factor of
// L = Lt D (Lt(r, c) = L(r, c) / L(c, c), D = diag(L)): forward Lt z = b
// (then y = D^-1 z), backward Lt^T x = D^-1 y = D^-2 z. A solve copy of the
// top levels' panels holds Lt row-major, each row padded to ws = w rounded
// up to 4 columns, with zeros on and above the diagonal of each diagonal
// block (k_solve_copy, once per factorization): a column step of either
// sweep is one lane broadcast and one FMA per entry held (no masks, no
// scaling on the chain); the forward sweep reads four columns of its row
// per LDS access, the backward sweep's column-per-lane reads are
// consecutive across lanes.
__host__ __device__ inline int tree2_ws(int w) { return (w + 3) & ~3; }

// four consecutive entries from a 16-byte aligned LDS address (FP32: one
// 128-bit read; FP64: two)
__device__ __forceinline__ void load4(float (&a)[4], const float* p) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    a[0] = t.x; a[1] = t.y; a[2] = t.z; a[3] = t.w;
}
__device__ __forceinline__ void load4(double (&a)[4], const double* p) {
    const double2 t0 = *reinterpret_cast<const double2*>(p);
    const double2 t1 = *reinterpret_cast<const double2*>(p + 2);
    a[0] = t0.x; a[1] = t0.y; a[2] = t1.x; a[3] = t1.y;
}

// forward sweep of one supernode (w columns, nr rows, staged panel at p0,
// first column at LDS slot `slot`, below-diagonal row slots at rsl[rs..]);
// leaves D^-2 z on the supernode's columns and adds the updates into the
// ancestors' entries
template <typename T, int R>
__device__ __forceinline__ void fwd2(int w, int nr, int slot, int rs, int p0, const T* P, T* xs, const T* dv,
                                     const i32* rsl) {
    constexpr int CH = tree2_chunk<T, R>();
    const int lane = threadIdx.x & (kWave - 1);
    const int ws = tree2_ws(w);
    T v[R];
    const T* Pr[R];   // row of the panel (lanes past nr: row nr - 1, never read back)
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int row = lane + kWave * r;
        const T a = xs[slot + min(row, w - 1)];
        v[r] = row < w ? a : T(0);
        Pr[r] = P + p0 + min(row, nr - 1) * ws;
    }
#pragma unroll
    for (int rb = 0; rb < R; rb++) {
        const int cend = min(w, kWave * (rb + 1));
        for (int c0 = kWave * rb; c0 < cend; c0 += CH) {
            // four columns per read; columns past w read as zero (padding
            // up to ws, masked beyond), so the column steps carry no guard
            T lc[CH][R];
#pragma unroll
            for (int r = 0; r < R; r++)
#pragma unroll
                for (int cc = 0; cc < CH; cc += 4)
                    if (r >= rb) {
                        const int cq = min(c0 + cc, ws - 4);
                        T a[4];
                        load4(a, Pr[r] + cq);
#pragma unroll
                        for (int u = 0; u < 4; u++) lc[cc + u][r] = c0 + cc < ws ? a[u] : T(0);
                    }
#pragma unroll
            for (int cc = 0; cc < CH; cc++) {
                const T zc = lane_read(v[rb], (c0 + cc) & (kWave - 1));   // final z_c
#pragma unroll
                for (int r = 0; r < R; r++)
                    if (r >= rb) v[r] -= lc[cc][r] * zc;   // rows above block rb take no update
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int row = lane + kWave * r;
        if (row < w) {
            const T e = dv[slot + row];
            xs[slot + row] = v[r] * e * e;
        } else if (row < nr) {
            atomicAdd(&xs[rsl[rs + row - w]], v[r]);
        }
    }
}

// backward sweep of one supernode; lane i holds diagonal-block column i
// (and i + 64, ... for wider supernodes): the solved rows below are folded
// in by per-lane dot products, then the triangle is swept from the last
// column down
template <typename T, int R>
__device__ __forceinline__ void bwd2(int w, int nr, int slot, int rs, int p0, const T* P, T* xs, const i32* rsl) {
    constexpr int CH = tree2_chunk<T, R>();
    const int lane = threadIdx.x & (kWave - 1);
    const int nb = nr - w, ws = tree2_ws(w);
    T acc[R], acc2[R], xb[R];
    const T* Pc[R];   // column i of the panel, stride ws (lanes past w: column w - 1, never read back)
#pragma unroll
    for (int q = 0; q < R; q++) {
        const int i = lane + kWave * q, ic = min(i, w - 1);
        const T a = xs[slot + ic];
        acc[q] = i < w ? a : T(0);
        acc2[q] = T(0);
        Pc[q] = P + p0 + ic;
        T xv = T(0);
        if (nb > 0) xv = xs[rsl[rs + min(i, nb - 1)]];
        xb[q] = i < nb ? xv : T(0);
    }
    // acc_i -= sum_k Lt(w + k, i) x(w + k), CH rows at a time
#pragma unroll
    for (int kb = 0; kb < R; kb++) {
        const int kend = min(nb - kWave * kb, kWave);
        for (int k0 = 0; k0 < kend; k0 += CH) {
            T pa[CH][R];
#pragma unroll
            for (int kk = 0; kk < CH; kk++) {
                const int row = w + kWave * kb + min(k0 + kk, kend - 1);
#pragma unroll
                for (int q = 0; q < R; q++) pa[kk][q] = Pc[q][row * ws];
            }
#pragma unroll
            for (int kk = 0; kk < CH; kk++) {
                // lanes past the last row below hold zero
                const T xr = lane_read(xb[kb], (k0 + kk) & (kWave - 1));
#pragma unroll
                for (int q = 0; q < R; q++) {
                    if (kk & 1) acc2[q] -= pa[kk][q] * xr;
                    else acc[q] -= pa[kk][q] * xr;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < R; q++) acc[q] += acc2[q];
    // the triangle, from the last column down
#pragma unroll
    for (int qb = R - 1; qb >= 0; qb--) {
        if (kWave * qb >= w) continue;
        const int jlo = kWave * qb;
        for (int j1 = min(w, kWave * (qb + 1)) - 1; j1 >= jlo; j1 -= CH) {
            // Lt(j, i), zero for j <= i; rows below jlo (the last chunk's
            // tail) read as zero, so the steps carry no guard
            T t[CH][R];
#pragma unroll
            for (int q = 0; q < R; q++)
#pragma unroll
                for (int jj = 0; jj < CH; jj++)
                    if (q <= qb) {
                        const T a = Pc[q][max(j1 - jj, jlo) * ws];
                        t[jj][q] = j1 - jj >= jlo ? a : T(0);
                    }
#pragma unroll
            for (int jj = 0; jj < CH; jj++) {
                const T xj = lane_read(acc[qb], (j1 - jj) & (kWave - 1));   // final x_j
#pragma unroll
                for (int q = 0; q < R; q++)
                    if (q <= qb) acc[q] -= t[jj][q] * xj;   // columns right of block qb are final
            }
        }
    }
#pragma unroll
    for (int q = 0; q < R; q++) {
        const int i = lane + kWave * q;
        if (i < w) xs[slot + i] = acc[q];
    }
}

// Packed solve copy of the wavefront solves' supernodes: entry e of an
// instance's copy is entry src[e] of its L storage (the map is built with
// the analysis). Instances whose active flag is clear are left as they are.
template <typename T, typename IX>
__global__ void k_pack(const IX* __restrict__ src, i64 np, const T* __restrict__ L, i64 Lsize, T* __restrict__ Lp,
                       const int* active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const T* Lb = L + (i64)b * Lsize;
    T* Pb = Lp + (i64)b * np;
    for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < np; e += (i64)gridDim.x * blockDim.x)
        Pb[e] = Lb[src[e]];
}

// Solve copy of the panels of supernodes desc[0, gridDim.x): row-major,
// rows of ws = tree2_ws(w) entries, Lt(r, c) = L(r, c) / L(c, c) below the
// diagonal, zero on and above it and in the padding, at offset toff - base
// of instance b's copy (ltsize entries per instance).
template <typename T>
__global__ void k_solve_copy(const TreeDesc* __restrict__ desc, const T* __restrict__ L, i64 Lsize,
                             const T* __restrict__ Dinv, i64 n, T* __restrict__ Lt, i64 ltsize, i64 base) {
    const TreeDesc d = desc[blockIdx.x];
    const int b = blockIdx.y;
    const int ws = tree2_ws(d.w);
    const T* src = L + (i64)b * Lsize + d.lptr;
    T* dst = Lt + (i64)b * ltsize + (d.toff - base);
    const T* di = Dinv + (i64)b * n + d.f;
    const int tot = d.nr * ws;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
        const int row = e / ws, c = e - row * ws;
        dst[e] = (c < d.w && row > c) ? src[(i64)c * d.nr + row] * di[c] : T(0);
    }
}

// forward over levels [l0, l1), then backward. tcols[0..nt) are the columns
// of those levels (slot i holds x[tcols[i]]); desc[lev_desc0[l0] ..
// lev_desc0[l1]) their supernodes, trs[rs0, rs0 + nrs) their row slots;
// level l's panels are the solve copy's [lev_off[l] - base, lev_off[l + 1]
// - base) (ltsize entries per instance), at most pmax <= NT * PR entries.
template <typename T, int NT, int PR>
__global__ __launch_bounds__(NT) void k_tri_tree2(SymView S, const TreeDesc* __restrict__ desc,
                                                  const i32* __restrict__ lev_desc0, const i64* __restrict__ lev_off,
                                                  int l0, int l1, const i32* __restrict__ tcols, int nt,
                                                  const i32* __restrict__ trs, int rs0, int nrs, int pmax,
                                                  const T* __restrict__ Lt, i64 ltsize, i64 base,
                                                  const T* __restrict__ Dinv, T* __restrict__ X, const int* ids,
                                                  const CGState* st) {
    extern __shared__ double smem_d[];
    const int nlev = l1 - l0;
    const int d0 = lev_desc0[l0], nd = lev_desc0[l1] - d0;
    const Tree2Lds o = tree2_layout(nt, (int)sizeof(T), nd, nrs, nlev, S.G, pmax);
    unsigned char* sm = reinterpret_cast<unsigned char*>(smem_d);
    T* xs = reinterpret_cast<T*>(sm + o.xs);
    T* dv = reinterpret_cast<T*>(sm + o.dv);
    TreeDesc* dl = reinterpret_cast<TreeDesc*>(sm + o.desc);
    i32* rsl = reinterpret_cast<i32*>(sm + o.rs);
    i32* lvd = reinterpret_cast<i32*>(sm + o.lvd);
    i64* lvp = reinterpret_cast<i64*>(sm + o.lvp);
    int* done = reinterpret_cast<int*>(sm + o.done);
    T* P = reinterpret_cast<T*>(sm + o.pan);
    const int b = inst_of(ids, blockIdx.x);
    T* x = X + (i64)b * S.n;
    const T* Lb = Lt + (i64)b * ltsize;
    const T* Db = Dinv + (i64)b * S.n;
    for (int i = threadIdx.x; i < nt; i += NT) {
        const int col = tcols[i];
        xs[i] = x[col];
        dv[i] = Db[col];
    }
    for (int i = threadIdx.x; i < nd; i += NT) {
        TreeDesc e = desc[d0 + i];
        e.rs -= rs0;
        dl[i] = e;
    }
    for (int i = threadIdx.x; i < nrs; i += NT) rsl[i] = trs[rs0 + i];
    for (int i = threadIdx.x; i <= nlev; i += NT) {
        lvd[i] = lev_desc0[l0 + i] - d0;
        lvp[i] = lev_off[l0 + i] - base;
    }
    for (int k = threadIdx.x; k < S.G; k += NT) done[k] = st ? st[(i64)b * S.G + k].done : 0;
    T pr[PR];
    tree2_load<T, PR>(pr, Lb + (lev_off[l0] - base), (int)(lev_off[l0 + 1] - lev_off[l0]), threadIdx.x, NT);
    const int wv = wave_in_block(), nw = NT / kWave;
    int lw = 0;   // first wavefront of the threads holding the next visit's panels
    // visits: levels l0 .. l1-1 forward, then l1-1 .. l0 backward; the top
    // level's staged panels serve both of its visits
    for (int v = 0; v < 2 * nlev; v++) {
        const bool fwd = v < nlev;
        const int li = fwd ? v : 2 * nlev - 1 - v;
        __syncthreads();   // previous visit done with P and xs
        if (v != nlev) {
            if (wv >= lw)
                tree2_store<T, PR>(pr, P, (int)(lvp[li + 1] - lvp[li]), threadIdx.x - lw * kWave, NT - lw * kWave);
            __syncthreads();
        }
        // the next visit's panels are loaded by the wavefronts without a
        // supernode in this visit when they can hold them, so the loads do
        // not hold up the ones that solve
        const int vn = v + 1;
        if (vn < 2 * nlev && vn != nlev) {
            const int ln = vn < nlev ? vn : 2 * nlev - 1 - vn;
            const int ne = (int)(lvp[ln + 1] - lvp[ln]);
            lw = min(lvd[li + 1] - lvd[li], nw);
            if (lw >= nw || (nw - lw) * kWave * PR < ne) lw = 0;
            if (wv >= lw) tree2_load<T, PR>(pr, Lb + lvp[ln], ne, threadIdx.x - lw * kWave, NT - lw * kWave);
        }
        const i64 pbase = lvp[li];
        for (int q = lvd[li] + wv; q < lvd[li + 1]; q += nw) {
            const TreeDesc& e = dl[q];
            const int w = __builtin_amdgcn_readfirstlane(e.w);
            const int nr = __builtin_amdgcn_readfirstlane(e.nr);
            const int slot = __builtin_amdgcn_readfirstlane(e.slot);
            const int rs = __builtin_amdgcn_readfirstlane(e.rs);
            const int p0 = __builtin_amdgcn_readfirstlane((int)(e.toff - base - pbase));
            if (__builtin_amdgcn_readfirstlane(done[e.mem])) continue;
            if (fwd) {
                if (nr <= kWave) fwd2<T, 1>(w, nr, slot, rs, p0, P, xs, dv, rsl);
                else if (nr <= 2 * kWave) fwd2<T, 2>(w, nr, slot, rs, p0, P, xs, dv, rsl);
                else fwd2<T, 4>(w, nr, slot, rs, p0, P, xs, dv, rsl);
            } else {
                if (nr <= kWave) bwd2<T, 1>(w, nr, slot, rs, p0, P, xs, rsl);
                else if (nr <= 2 * kWave) bwd2<T, 2>(w, nr, slot, rs, p0, P, xs, rsl);
                else bwd2<T, 4>(w, nr, slot, rs, p0, P, xs, rsl);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nt; i += NT) x[tcols[i]] = xs[i];
}

// one class per launch (used for the wide classes R >= 4)
template <typename T, int SEG, int R, bool PUSH>
__global__ __launch_bounds__(kBlock) void k_fwd_s(SymView S, const TriDesc* __restrict__ desc, int count, int npad,
                                                  const T* __restrict__ Lp, const T* __restrict__ Dinv,
                                                  T* __restrict__ X, T* __restrict__ UV, const int* ids, int nids,
                                                  const CGState* st) {
    fwd_task<T, SEG, R, PUSH>(S, desc, count, npad, (i64)blockIdx.x * (kBlock / kWave) + wave_in_block(), Lp, Dinv,
                              X, UV, ids, nids, st);
}

template <typename T, int SEG, int R>
__global__ __launch_bounds__(kBlock) void k_bwd_s(SymView S, const TriDesc* __restrict__ desc, int count, int npad,
                                                  const T* __restrict__ Lp, const T* __restrict__ Dinv,
                                                  T* __restrict__ X, const int* ids, int nids, const CGState* st) {
    bwd_task<T, SEG, R>(S, desc, count, npad, (i64)blockIdx.x * (kBlock / kWave) + wave_in_block(), Lp, Dinv, X,
                        ids, nids, st);
}

// the four narrow classes of one level in one launch: each wavefront looks
// up its class by the wavefront ranges and runs that class's task
struct LevelTasks {
    const TriDesc* desc[4];
    int count[4];
    int npad[4];
    i64 wave_end[4];   // cumulative wavefront counts
};

template <typename T, bool PUSH>
__global__ __launch_bounds__(kBlock) void k_fwd_lvl(SymView S, LevelTasks lt, const T* __restrict__ Lp,
                                                    const T* __restrict__ Dinv, T* __restrict__ X, T* __restrict__ UV,
                                                    const int* ids, int nids, const CGState* st) {
    const i64 wv = (i64)blockIdx.x * (kBlock / kWave) + wave_in_block();
    if (wv < lt.wave_end[0])
        fwd_task<T, 16, 1, PUSH>(S, lt.desc[0], lt.count[0], lt.npad[0], wv, Lp, Dinv, X, UV, ids, nids, st);
    else if (wv < lt.wave_end[1])
        fwd_task<T, 32, 1, PUSH>(S, lt.desc[1], lt.count[1], lt.npad[1], wv - lt.wave_end[0], Lp, Dinv, X, UV, ids, nids, st);
    else if (wv < lt.wave_end[2])
        fwd_task<T, 64, 1, PUSH>(S, lt.desc[2], lt.count[2], lt.npad[2], wv - lt.wave_end[1], Lp, Dinv, X, UV, ids, nids, st);
    else if (wv < lt.wave_end[3])
        fwd_task<T, 64, 2, PUSH>(S, lt.desc[3], lt.count[3], lt.npad[3], wv - lt.wave_end[2], Lp, Dinv, X, UV, ids, nids, st);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bwd_lvl(SymView S, LevelTasks lt, const T* __restrict__ Lp,
                                                    const T* __restrict__ Dinv, T* __restrict__ X, const int* ids,
                                                    int nids, const CGState* st) {
    const i64 wv = (i64)blockIdx.x * (kBlock / kWave) + wave_in_block();
    if (wv < lt.wave_end[0])
        bwd_task<T, 16, 1>(S, lt.desc[0], lt.count[0], lt.npad[0], wv, Lp, Dinv, X, ids, nids, st);
    else if (wv < lt.wave_end[1])
        bwd_task<T, 32, 1>(S, lt.desc[1], lt.count[1], lt.npad[1], wv - lt.wave_end[0], Lp, Dinv, X, ids, nids, st);
    else if (wv < lt.wave_end[2])
        bwd_task<T, 64, 1>(S, lt.desc[2], lt.count[2], lt.npad[2], wv - lt.wave_end[1], Lp, Dinv, X, ids, nids, st);
    else if (wv < lt.wave_end[3])
        bwd_task<T, 64, 2>(S, lt.desc[3], lt.count[3], lt.npad[3], wv - lt.wave_end[2], Lp, Dinv, X, ids, nids, st);
}

// ---------------------------------------------------------------------------
// Dataflow triangular solves: the forward sweep over every level and then
// the backward sweep, for all listed instances, in one launch. The wave
// tasks (one supernode descriptor x a group of 64/SEG instance slots, as in
// the per-level kernels) are numbered forward levels up, then backward
// levels down, classes 0..3 within a level; wave w takes tasks w, w + W, ...
// in that order. A task needs no level barrier: it issues its panel and
// diagonal loads, waits (one lane per segment polling) until its own
// dependencies are met, acquires, solves and releases:
//   forward (b, s): all children of s have added their updates into x
//     (fcnt[b][s] == nchild; the task then clears its counter), then adds
//     its own rows below into the ancestors' entries (FP atomics) and counts
//     itself done at its parent (or marks fflag = app at a root);
//   backward (b, s): the parent's backward task is done (bflag[b][parent]
//     == app; a root waits for its own forward task), then marks bflag.
// A child is done only after its own children, so "all children done"
// covers every descendant that updates x at the columns of s. Tasks are
// assigned in a topological order and every wait is on an earlier task, so
// the launch completes when its work-groups are co-resident (the grid is
// sized to a fraction of the device); every wait is also bounded: after
// kFlowSpin polls it sets *abort and every later wait returns, so the
// launch always ends (the host then reports the failure).
// ---------------------------------------------------------------------------
constexpr int kFlowSpin = 1 << 20;

__device__ __forceinline__ void flow_wait(const int* p, int target, bool need, int* abortf) {
    bool ok = !need;
    int spins = 0;
    while (true) {
        if (!ok) ok = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == target;
        if (__all(ok)) break;
        if (__hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        if (++spins > kFlowSpin) {
            __hip_atomic_store(abortf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <typename T, int SEG, int R>
__device__ __forceinline__ void flow_fwd(const SymView& S, const FlowArgs& F, const TriDesc& d, int qi, int b,
                                         bool valid, const T* __restrict__ L, const T* __restrict__ Dinv,
                                         T* __restrict__ X) {
    constexpr int CH = chunk_cols<T, SEG, R>();
    const int sl = threadIdx.x & (SEG - 1);
    const T* Lb = L + (i64)b * S.Lsize + d.lptr;
    const T* dinv = Dinv + (i64)b * S.n + d.f;
    T* x = X + (i64)b * S.n;
    T lc[CH][R];
    load_cols<T, SEG, R, CH, false>(lc, Lb, d, 0, sl);     // the factor is not written during the solve
    T di[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int row = sl + SEG * r;
        di[r] = row < d.w ? dinv[row] : T(0);
    }
    int* cnt = F.fcnt + (i64)b * F.ndesc + qi;
    const bool lead = valid && sl == 0;
    flow_wait(cnt, d.nchild, lead && d.nchild > 0, F.abort);
    if (lead && d.nchild > 0) __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    T v[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int row = sl + SEG * r;
        v[r] = row < d.w ? x[d.f + row] : T(0);
    }
    fwd_cols<T, SEG, R, CH, true, false>(lc, v, di, Lb, d, sl);
    if (valid) {
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int row = sl + SEG * r;
            if (row < d.w) x[d.f + row] = v[r];
            else if (row < d.nr) unsafeAtomicAdd(&x[S.sn_rows[d.rp + row]], v[r]);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lead) {
        if (d.pq >= 0)
            __hip_atomic_fetch_add(F.fcnt + (i64)b * F.ndesc + d.pq, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            __hip_atomic_store(F.fflag + (i64)b * F.ndesc + qi, F.app, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename T, int SEG, int R>
__device__ __forceinline__ void flow_bwd(const SymView& S, const FlowArgs& F, const TriDesc& d, int qi, int b,
                                         bool valid, const T* __restrict__ L, const T* __restrict__ Dinv,
                                         T* __restrict__ X) {
    constexpr int CH = chunk_cols<T, SEG, R>();
    const int sl = threadIdx.x & (SEG - 1);
    const T* Lb = L + (i64)b * S.Lsize + d.lptr;
    const T* dinv = Dinv + (i64)b * S.n + d.f;
    T* x = X + (i64)b * S.n;
    T lc[CH][R];
    load_cols<T, SEG, R, CH, false>(lc, Lb, d, d.w - CH, sl);
    T di[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int row = sl + SEG * r;
        di[r] = row < d.w ? dinv[row] : T(0);
    }
    const int* dep = d.pq < 0 ? F.fflag + (i64)b * F.ndesc + qi : F.bflag + (i64)b * F.ndesc + d.pq;
    flow_wait(dep, F.app, valid && sl == 0, F.abort);
    T v[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int row = sl + SEG * r;
        T a = T(0);
        if (row < d.nr) a = row < d.w ? x[d.f + row] : x[S.sn_rows[d.rp + row]];
        v[r] = a;
    }
    bwd_cols<T, SEG, R, CH, true, false>(lc, v, di, Lb, d, sl);
    if (valid) {
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int row = sl + SEG * r;
            if (row < d.w) x[d.f + row] = v[r];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (valid && sl == 0)
        __hip_atomic_store(F.bflag + (i64)b * F.ndesc + qi, F.app, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, int SEG, int R>
__device__ __forceinline__ void flow_task(const SymView& S, const FlowArgs& F, const TriDesc* __restrict__ desc,
                                          bool fwd, int off, i64 u, const T* __restrict__ L,
                                          const T* __restrict__ Dinv, T* __restrict__ X) {
    constexpr int G = kWave / SEG;
    const int ng = (F.nids + G - 1) / G;
    const int q = (int)(u / ng);
    const int k = (int)(u - (i64)q * ng) * G + (int)(threadIdx.x & (kWave - 1)) / SEG;
    bool valid = k < F.nids;
    const int b = valid ? inst_of(F.ids, k) : inst_of(F.ids, 0);
    const int qi = off + q;
    const TriDesc d = desc[qi];
    if (valid && F.st && F.st[(i64)b * S.G + d.mem].done) valid = false;
    if (fwd) flow_fwd<T, SEG, R>(S, F, d, qi, b, valid, L, Dinv, X);
    else flow_bwd<T, SEG, R>(S, F, d, qi, b, valid, L, Dinv, X);
}

__host__ __device__ constexpr int flow_group(int cls) { return cls == 0 ? 4 : cls == 1 ? 2 : 1; }

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tri_flow(SymView S, FlowArgs F, const TriDesc* __restrict__ desc,
                                                     const T* __restrict__ L, const T* __restrict__ Dinv,
                                                     T* __restrict__ X) {
    const i64 W = (i64)gridDim.x * (kBlock / kWave);
    const i64 wave = (i64)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int nseg = 2 * F.nlevels * 4;
    int si = 0;
    i64 s0 = 0;   // first task of segment si
    auto seg_of = [&](int i, bool* fwd, int* cls, int* off, int* cnt) {
        const int half = F.nlevels * 4;
        *fwd = i < half;
        const int j = *fwd ? i : i - half;
        const int lv = *fwd ? j / 4 : F.nlevels - 1 - j / 4;
        *cls = j % 4;
        *off = F.seg[2 * (lv * kTriClasses + *cls)];
        *cnt = F.seg[2 * (lv * kTriClasses + *cls) + 1];
    };
    for (i64 t = wave;; t += W) {
        bool fwd = true;
        int cls = 0, off = 0, cnt = 0;
        while (si < nseg) {
            seg_of(si, &fwd, &cls, &off, &cnt);
            const i64 len = (i64)cnt * ((F.nids + flow_group(cls) - 1) / flow_group(cls));
            if (t < s0 + len) break;
            s0 += len;
            si++;
        }
        if (si >= nseg) return;
        const i64 u = t - s0;
        switch (cls) {
            case 0: flow_task<T, 16, 1>(S, F, desc, fwd, off, u, L, Dinv, X); break;
            case 1: flow_task<T, 32, 1>(S, F, desc, fwd, off, u, L, Dinv, X); break;
            case 2: flow_task<T, 64, 1>(S, F, desc, fwd, off, u, L, Dinv, X); break;
            default: flow_task<T, 64, 2>(S, F, desc, fwd, off, u, L, Dinv, X); break;
        }
    }
}

// reciprocals of the factor's diagonal (one per column), used by the
// wavefront triangular solves in place of divisions
template <typename T>
__global__ void k_inv_diag(const i64* __restrict__ diag_off, i64 n, i64 Lsize, const T* __restrict__ L,
                           T* __restrict__ Dinv, const int* active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    for (i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (i64)gridDim.x * blockDim.x)
        Dinv[(i64)b * n + j] = T(1) / L[(i64)b * Lsize + diag_off[j]];
}

// ---------------------------------------------------------------------------
// SpMV with J^T (rows = permuted columns of J):
//   out[b][i] = a[b][i] + scale * g * sum_k JT[b][k] * v[b][JT_col[k]]
// with g = gamma of the row's member if use_gamma else 1; a may be null.
// Rows of members whose CG is done (st) are left alone.
// ---------------------------------------------------------------------------
// Dot product of CSR row entries [k0, k1) with a gathered vector, in entry
// order (the same sum as a plain loop), with the index and value loads of
// eight entries and then their eight gathers in flight at once instead of
// one dependent gather per entry.
template <typename TV>
__device__ __forceinline__ double row_dot(i64 k0, i64 k1, const double* __restrict__ val,
                                          const i32* __restrict__ col, const TV* __restrict__ x) {
    double sum = 0.0;
    for (i64 k = k0; k < k1; k += 8) {
        double vv[8];
        i32 cc[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const i64 kk = k + u < k1 ? k + u : k1 - 1;
            vv[u] = val[kk];
            cc[u] = col[kk];
        }
        TV xv[8];
#pragma unroll
        for (int u = 0; u < 8; u++) xv[u] = x[cc[u]];
#pragma unroll
        for (int u = 0; u < 8; u++)
            if (k + u < k1) sum += vv[u] * (double)xv[u];
    }
    return sum;
}

template <typename TO>
__global__ void k_jt(SymView S, ValView V, const double* __restrict__ a, double scale, int use_gamma,
                     const double* __restrict__ v, TO* __restrict__ out, const int* ids, const CGState* st) {
    const int b = inst_of(ids, blockIdx.y);
    const double* JT = V.JT + (i64)b * S.nnzJ;
    const double* vb = v + (i64)b * S.m;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < S.n; i += (i64)gridDim.x * blockDim.x) {
        // the convergence flag only gates the store: its load overlaps the others
        const i64 c = (i64)b * S.G + mem_x(S, i);
        const bool done = st && st[c].done;
        const double sc = scale * (use_gamma ? V.gamma[c] : 1.0);
        const double sum = row_dot(S.JT_rowptr[i], S.JT_rowptr[i + 1], JT, S.JT_col, vb);
        const double base = a ? a[(i64)b * S.n + i] : 0.0;
        if (!done) out[(i64)b * S.n + i] = (TO)(base + sc * sum);
    }
}

// Member-aligned blocks: block j of a table covers indices [t[3j], t[3j+1])
// of member t[3j+2]; every block holds at most kBlock indices, so one
// work-group of kBlock threads takes one block. Partial sums of batch entry b
// go to part[b * nblk + j] and are reduced per member over the member's
// consecutive blocks.
struct Blk {
    i64 lo, hi;
    int k;
};
__device__ __forceinline__ Blk blk_of(const i32* t, int j) { return {t[3 * j], t[3 * j + 1], t[3 * j + 2]}; }

// SpMV with J (permuted columns), FP64 accumulation of an FP32 or FP64 input,
// over the member-aligned blocks of the J rows (grid.x = S.nbm).
// mode 0 (Schur right-hand side): q = J u - sub; part1 = sum q^2.
// mode 1 (CG): q = J u + d2 * p; part1 = sum p.q; part2 = sum p.p.
template <typename TI>
__global__ __launch_bounds__(kBlock) void k_j(SymView S, ValView V, const TI* __restrict__ u, const double* __restrict__ sub,
                                              const double* __restrict__ p, const CGState* st, int mode,
                                              double* __restrict__ q, double* __restrict__ part1,
                                              double* __restrict__ part2, const int* ids) {
    __shared__ double sh[kBlock / kWave];
    const int b = inst_of(ids, blockIdx.y);
    const Blk bk = blk_of(S.mblk, blockIdx.x);
    const i64 c = (i64)b * S.G + bk.k;
    // the convergence flag (uniform in the block) only gates the stores: its
    // load overlaps the row's loads
    const bool done = mode == 1 && st[c].done;
    const double* J = V.J + (i64)b * S.nnzJ;
    const TI* ub = u + (i64)b * S.n;
    const i64 i = bk.lo + threadIdx.x;
    double a1 = 0.0, a2 = 0.0;
    if (i < bk.hi) {
        double sum = row_dot(S.J_rowptr[i], S.J_rowptr[i + 1], J, S.J_colp, ub);
        if (mode == 0) {
            sum -= sub[(i64)b * S.m + i];
            a1 = sum * sum;
        } else {
            const double pi = p[(i64)b * S.m + i];
            sum += st[c].d2 * pi;
            a1 = pi * sum;
            a2 = pi * pi;
        }
        if (!done) q[(i64)b * S.m + i] = sum;
    }
    if (done) return;   // uniform in the block
    a1 = block_sum(a1, sh);
    if (mode == 1) a2 = block_sum(a2, sh);
    if (threadIdx.x == 0) {
        part1[(i64)b * gridDim.x + blockIdx.x] = a1;
        if (mode == 1) part2[(i64)b * gridDim.x + blockIdx.x] = a2;
    }
}

// ---------------------------------------------------------------------------
// CG on S y = bvec (unpreconditioned, y0 = 0), Algorithm 1 / eq. Schur1, one
// independent CG per (batch entry, member). Scalar kernels: grid.x = list
// index, grid.y = member.
// ---------------------------------------------------------------------------
__device__ double reduce_parts(const double* part, int nblk, double* sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) v += part[i];
    return block_sum(v, sh);
}

// sum of the partials of member k of batch entry b
__device__ __forceinline__ double reduce_member(const double* part, int nblk, const i32* off, int b, int k,
                                                double* sh) {
    return reduce_parts(part + (i64)b * nblk + off[k], off[k + 1] - off[k], sh);
}

// rho = ||b||^2, reset the state; members not in this pass (cact) start done
__global__ void k_cg_init(SymView S, CGState* st, const double* part, const int* ids, const int* cact) {
    __shared__ double sh[kBlock / kWave];
    const int b = inst_of(ids, blockIdx.x), k = blockIdx.y;
    const i64 ci = (i64)b * S.G + k;
    const double r = reduce_member(part, S.nbm, S.mblk_off, b, k, sh);
    if (threadIdx.x == 0) {
        CGState c = {};
        c.rho = r;
        c.bnorm = sqrt(r);
        c.curv0 = -1.0;
        c.done = (cact && !cact[ci]) || !(r > 0.0);
        st[ci] = c;
    }
}

__global__ void k_cg_vecinit(const double* __restrict__ bvec, double* __restrict__ y, double* __restrict__ res,
                             double* __restrict__ p, i64 m, const int* ids) {
    const int b = inst_of(ids, blockIdx.y);
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (i64)gridDim.x * blockDim.x) {
        const double v = bvec[(i64)b * m + i];
        y[(i64)b * m + i] = 0.0;
        res[(i64)b * m + i] = v;
        p[(i64)b * m + i] = v;
    }
}

// alpha = rho / p'q, with the small-quadratic-form test of Algorithm 1
// (on the state of a member whose CG is running)
__device__ __forceinline__ void cg_alpha_step(CGState& c, double pq, double pp, double qf_eps, double delta2) {
    if (c.curv0 < 0.0) c.curv0 = pq / pp;
    c.pq = pq;
    c.pp = pp;
    if (!(pq > qf_eps * pp * c.curv0)) {
        c.breakdown = 1;
        if (delta2 > 0.0 && c.d2 == 0.0) {
            c.d2 = delta2;      // restart on S + delta2 I
            c.alpha = 0.0;
            c.pad = 1;          // restart pending
        } else {
            c.done = 1;
        }
    } else {
        c.alpha = c.rho / pq;
    }
}

// y += alpha p; res -= alpha q; partial res'res into part (member-aligned
// blocks of the J rows). Every block forms alpha itself from the state at the
// start of the iteration and the p'q, p'p partials (part1, part2), by the
// same reduction as k_cg_beta, which stores the state afterwards: the state
// is read-only here. A pending restart resets y = 0, res = bvec.
__global__ __launch_bounds__(kBlock) void k_cg_update(SymView S, const double* __restrict__ p,
                                                      const double* __restrict__ q, const double* __restrict__ bvec,
                                                      double* __restrict__ y, double* __restrict__ res,
                                                      const CGState* st, const double* part1, const double* part2,
                                                      double qf_eps, double delta2, double* __restrict__ part,
                                                      const int* ids) {
    __shared__ double sh[kBlock / kWave];
    const int b = inst_of(ids, blockIdx.y);
    const Blk bk = blk_of(S.mblk, blockIdx.x);
    // the state (uniform in the block) and the vectors are loaded before the
    // reductions' barriers
    CGState c = st[(i64)b * S.G + bk.k];
    const i64 i = bk.lo + threadIdx.x;
    const bool in = i < bk.hi;
    const i64 o = (i64)b * S.m + i;
    double pv = 0.0, qv = 0.0, yv = 0.0, rv = 0.0, bv = 0.0;
    if (in) {
        pv = p[o];
        qv = q[o];
        yv = y[o];
        rv = res[o];
        bv = bvec[o];
    }
    // the block sums are complete in thread 0 only: it hands them to the others
    __shared__ double pqpp[2];
    const double pq0 = reduce_member(part1, S.nbm, S.mblk_off, b, bk.k, sh);
    const double pp0 = reduce_member(part2, S.nbm, S.mblk_off, b, bk.k, sh);
    if (threadIdx.x == 0) {
        pqpp[0] = pq0;
        pqpp[1] = pp0;
    }
    __syncthreads();
    if (!c.done) cg_alpha_step(c, pqpp[0], pqpp[1], qf_eps, delta2);
    if (c.done) return;   // uniform in the block
    double a = 0.0;
    if (in) {
        const double r = c.pad ? bv : rv - c.alpha * qv;
        y[o] = c.pad ? 0.0 : yv + c.alpha * pv;
        res[o] = r;
        a = r * r;
    }
    a = block_sum(a, sh);
    if (threadIdx.x == 0) part[(i64)b * gridDim.x + blockIdx.x] = a;
}

// the alpha step (as k_cg_update formed it) and then beta = r'r / rho with
// the convergence test; stores the state of the iteration
__global__ void k_cg_beta(SymView S, CGState* st, const double* part1, const double* part2, double qf_eps,
                          double delta2, const double* part, double tol, const double* ptol, int max_it,
                          const int* ids) {
    __shared__ double sh[kBlock / kWave];
    const int b = inst_of(ids, blockIdx.x), k = blockIdx.y;
    const i64 ci = (i64)b * S.G + k;
    const int done = st[ci].done;
    const double pq = reduce_member(part1, S.nbm, S.mblk_off, b, k, sh);
    const double pp = reduce_member(part2, S.nbm, S.mblk_off, b, k, sh);
    const double r1 = reduce_member(part, S.nbm, S.mblk_off, b, k, sh);
    if (done) return;   // uniform in the block
    if (threadIdx.x == 0) {
        CGState c = st[ci];
        cg_alpha_step(c, pq, pp, qf_eps, delta2);
        if (c.done) {
            // breakdown without a restart: y and res were left as they were
        } else if (c.pad) {
            c.pad = 0;
            c.rho = r1;
            c.beta = 0.0;
            c.curv0 = -1.0;
        } else {
            c.it++;
            const double t = ptol ? ptol[ci] : tol;   // per (instance, member) when given
            if (sqrt(r1) <= t * c.bnorm || c.it >= max_it) c.done = 1;
            c.beta = r1 / c.rho;
            c.rho = r1;
        }
        st[ci] = c;
    }
}

// p = res + beta p (member-aligned blocks of the J rows)
__global__ void k_cg_p(SymView S, double* __restrict__ p, const double* __restrict__ res, const CGState* st,
                       const int* ids) {
    const int b = inst_of(ids, blockIdx.y);
    const Blk bk = blk_of(S.mblk, blockIdx.x);
    const CGState* cs = st + (i64)b * S.G + bk.k;
    const int done = cs->done;
    const double be = cs->beta;
    const i64 i = bk.lo + threadIdx.x;
    if (i < bk.hi) {
        const i64 o = (i64)b * S.m + i;
        const double v = res[o] + be * p[o];
        if (!done) p[o] = v;
    }
}

// Order-preserving compaction of the batch entries with a member whose CG is
// still running (one work-group): ids_out = [b in ids_in live], *n_out = count.
__global__ void k_compact_live(const CGState* st, int G, const int* ids_in, int n_in, int* ids_out, int* n_out) {
    __shared__ int sc[kBlock];
    __shared__ int base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int c0 = 0; c0 < n_in; c0 += blockDim.x) {
        const int k = c0 + threadIdx.x;
        const int b = k < n_in ? ids_in[k] : -1;
        int f = 0;
        for (int g = 0; b >= 0 && g < G && !f; g++) f = !st[(i64)b * G + g].done;
        sc[threadIdx.x] = f;
        __syncthreads();
        for (int o = 1; o < (int)blockDim.x; o <<= 1) {
            const int v = threadIdx.x >= (unsigned)o ? sc[threadIdx.x - o] : 0;
            __syncthreads();
            sc[threadIdx.x] += v;
            __syncthreads();
        }
        if (f) ids_out[base + sc[threadIdx.x] - 1] = b;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) base += sc[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_out = base;
}

// ---------------------------------------------------------------------------
// refinement support (FP64), over the member-aligned blocks of the combined
// index space [x (n) ; y (m)] (grid.x = S.nbr)
// ---------------------------------------------------------------------------
// z += e for the members in this pass (cact; null: all)
__global__ __launch_bounds__(kBlock) void k_axpy2(SymView S, double* __restrict__ xz, const double* __restrict__ ex,
                                                  double* __restrict__ yz, const double* __restrict__ ey,
                                                  const int* ids, const int* cact) {
    const int b = inst_of(ids, blockIdx.y);
    const Blk bk = blk_of(S.rblk, blockIdx.x);
    if (cact && !cact[(i64)b * S.G + bk.k]) return;
    const i64 i = bk.lo + threadIdx.x;
    if (i >= bk.hi) return;
    if (i < S.n) xz[(i64)b * S.n + i] += ex[(i64)b * S.n + i];
    else yz[(i64)b * S.m + (i - S.n)] += ey[(i64)b * S.m + (i - S.n)];
}

// Compensated accumulation of r_i - sum_k a_k b_k (Ogita, Rump and Oishi
// 2005, "Accurate sum and dot product", Dot2): the running sum is the
// unevaluated pair hi + lo; each product is split exactly into p + ep by an
// FMA (TwoProduct) and hi - p exactly into s + es (TwoSum), and both error
// terms go to lo. The rounded result hi + lo is as accurate as a sum in
// twice the working precision. Contraction is off so that every product and
// sum is rounded on its own, as the transformations require.
struct Acc2 {
    double hi, lo, aabs;   // aabs: sum of |a_k b_k| (the evaluation floor's terms)
};

__device__ __forceinline__ void acc2_sub_prod(Acc2& c, double a, double b) {
#pragma clang fp contract(off)
    const double p = a * b;
    const double ep = __builtin_fma(a, b, -p);
    const double s = c.hi - p;
    const double z = s - c.hi;
    const double es = (c.hi - (s - z)) + (-p - z);
    c.hi = s;
    c.lo += es - ep;
    c.aabs += fabs(p);
}

// g = r - K z over rows [0, n) (first block row) and [n, n+m) (J rows),
// K = [H + D_x + delta I, J^T; J, 0], every product of a stored value with
// an entry of z a term of its own (the diagonal's H_ii, D_i and delta
// separately), summed by the compensated accumulation above; partial
// ||g||^2; optional partials of (|r_i| + sum of |term|)^2 (the floor:
// plain FP64 evaluation would err by about u times that).
__global__ __launch_bounds__(kBlock) void k_residual(SymView S, ValView V, const double* __restrict__ r1,
                                                     const double* __restrict__ r2, const double* __restrict__ xz,
                                                     const double* __restrict__ yz, double* __restrict__ g1,
                                                     double* __restrict__ g2, double* __restrict__ part,
                                                     double* __restrict__ part_floor, const int* ids) {
    __shared__ double sh[kBlock / kWave];
    const int b = inst_of(ids, blockIdx.y);
    const Blk bk = blk_of(S.rblk, blockIdx.x);
    const i64 i = bk.lo + threadIdx.x;
    const double* x = xz + (i64)b * S.n;
    const double* y = yz + (i64)b * S.m;
    double a = 0.0, fl = 0.0;
    if (i < bk.hi && i < S.n) {
        const double* HF = V.HF + (i64)b * S.nnzHF;
        const double* JT = V.JT + (i64)b * S.nnzJ;
        const double rv = r1[(i64)b * S.n + i];
        Acc2 c{rv, 0.0, 0.0};
        for (i64 k = S.HF_rowptr[i]; k < S.HF_rowptr[i + 1]; k++) acc2_sub_prod(c, HF[k], x[S.HF_col[k]]);
        const double xi = x[i];
        acc2_sub_prod(c, V.Dxp[(i64)b * S.n + i], xi);
        acc2_sub_prod(c, V.delta[(i64)b * S.G + bk.k], xi);
        for (i64 k = S.JT_rowptr[i]; k < S.JT_rowptr[i + 1]; k++) acc2_sub_prod(c, JT[k], y[S.JT_col[k]]);
        const double g = c.hi + c.lo;
        g1[(i64)b * S.n + i] = g;
        a = g * g;
        fl = c.aabs + fabs(rv);
        fl = fl * fl;
    } else if (i < bk.hi) {
        const i64 r = i - S.n;
        const double* J = V.J + (i64)b * S.nnzJ;
        const double rv = r2[(i64)b * S.m + r];
        Acc2 c{rv, 0.0, 0.0};
        for (i64 k = S.J_rowptr[r]; k < S.J_rowptr[r + 1]; k++) acc2_sub_prod(c, J[k], x[S.J_colp[k]]);
        const double g = c.hi + c.lo;
        g2[(i64)b * S.m + r] = g;
        a = g * g;
        fl = c.aabs + fabs(rv);
        fl = fl * fl;
    }
    a = block_sum(a, sh);
    if (part_floor) fl = block_sum(fl, sh);
    if (threadIdx.x == 0) {
        part[(i64)b * gridDim.x + blockIdx.x] = a;
        if (part_floor) part_floor[(i64)b * gridDim.x + blockIdx.x] = fl;
    }
}

// partial sums of squares of [v1 (n) ; v2 (m)] per block, all batch entries
__global__ __launch_bounds__(kBlock) void k_sumsq2(SymView S, const double* __restrict__ v1,
                                                   const double* __restrict__ v2, double* __restrict__ part) {
    __shared__ double sh[kBlock / kWave];
    const int b = blockIdx.y;
    const Blk bk = blk_of(S.rblk, blockIdx.x);
    const i64 i = bk.lo + threadIdx.x;
    double a = 0.0;
    if (i < bk.hi) a = i < S.n ? v1[(i64)b * S.n + i] : v2[(i64)b * S.m + (i - S.n)];
    a = block_sum(a * a, sh);
    if (threadIdx.x == 0) part[(i64)b * gridDim.x + blockIdx.x] = a;
}

// out[b * G + k] = sum of the partials of member k (grid.x = list index,
// grid.y = member; off = first block of each member)
__global__ void k_reduce_rows(const double* part, int nblk, const i32* off, double* out, const int* ids) {
    __shared__ double sh[kBlock / kWave];
    const int b = inst_of(ids, blockIdx.x), k = blockIdx.y;
    const double r = reduce_member(part, nblk, off, b, k, sh);
    if (threadIdx.x == 0) out[(i64)b * gridDim.y + k] = r;
}

// ||K||_inf per member: max row sum of |K| (Sec. 5.1 estimate of ||K||_2)
__global__ __launch_bounds__(kBlock) void k_knorm_rows(SymView S, ValView V, double* __restrict__ part) {
    __shared__ double sh[kBlock / kWave];
    const int b = blockIdx.y;
    const Blk bk = blk_of(S.rblk, blockIdx.x);
    const i64 i = bk.lo + threadIdx.x;
    double a = 0.0;
    if (i < bk.hi && i < S.n) {
        const double* HF = V.HF + (i64)b * S.nnzHF;
        const double* JT = V.JT + (i64)b * S.nnzJ;
        double dsum = V.Dxp[(i64)b * S.n + i] + V.delta[(i64)b * S.G + bk.k];
        for (i64 k = S.HF_rowptr[i]; k < S.HF_rowptr[i + 1]; k++) {
            if (S.HF_col[k] == i) dsum += HF[k];
            else a += fabs(HF[k]);
        }
        a += fabs(dsum);
        for (i64 k = S.JT_rowptr[i]; k < S.JT_rowptr[i + 1]; k++) a += fabs(JT[k]);
    } else if (i < bk.hi) {
        const i64 r = i - S.n;
        const double* J = V.J + (i64)b * S.nnzJ;
        for (i64 k = S.J_rowptr[r]; k < S.J_rowptr[r + 1]; k++) a += fabs(J[k]);
    }
    // block max
    for (int o = kWave / 2; o > 0; o >>= 1) a = fmax(a, __shfl_down(a, o, kWave));
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int t = 0; t < (int)(blockDim.x / kWave); t++) r = fmax(r, sh[t]);
        part[(i64)b * gridDim.x + blockIdx.x] = r;
    }
}

// ---------------------------------------------------------------------------
// quality check of a low-precision factor M: v is a fixed probe vector, w =
// M^{-1} v (the factor's own solve), t = J w; partial sums of
// (v - H_gamma w)^2 and v^2 over the x rows of the member-aligned blocks
// (H_gamma w = H w + (D_x + delta) w + gamma J^T (J w)).
// ---------------------------------------------------------------------------
__global__ void k_probe_vec(double* __restrict__ v, i64 n) {
    const int b = blockIdx.y;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        const unsigned h = (unsigned)(i * 2654435761ull) ^ (unsigned)(b * 40503u);
        v[(i64)b * n + i] = 0.5 + (double)(h >> 8) * (1.0 / 16777216.0);   // in [0.5, 1.5)
    }
}

template <typename TW>
__global__ __launch_bounds__(kBlock) void k_hgamma_check(SymView S, ValView V, const double* __restrict__ v,
                                                         const TW* __restrict__ w, const double* __restrict__ t,
                                                         double* __restrict__ part_r, double* __restrict__ part_v) {
    __shared__ double sh[kBlock / kWave];
    const int b = blockIdx.y;
    const Blk bk = blk_of(S.rblk, blockIdx.x);
    const i64 i = bk.lo + threadIdx.x;
    double a = 0.0, c = 0.0;
    if (i < bk.hi && i < S.n) {
        const double* HF = V.HF + (i64)b * S.nnzHF;
        const double* JT = V.JT + (i64)b * S.nnzJ;
        const TW* wb = w + (i64)b * S.n;
        const double* tb = t + (i64)b * S.m;
        double acc = 0.0, jt = 0.0;
        for (i64 k = S.HF_rowptr[i]; k < S.HF_rowptr[i + 1]; k++) acc += HF[k] * (double)wb[S.HF_col[k]];
        acc += (V.Dxp[(i64)b * S.n + i] + V.delta[(i64)b * S.G + bk.k]) * (double)wb[i];
        for (i64 k = S.JT_rowptr[i]; k < S.JT_rowptr[i + 1]; k++) jt += JT[k] * tb[S.JT_col[k]];
        acc += V.gamma[(i64)b * S.G + bk.k] * jt;
        const double vi = v[(i64)b * S.n + i];
        a = (vi - acc) * (vi - acc);
        c = vi * vi;
    }
    a = block_sum(a, sh);
    c = block_sum(c, sh);
    if (threadIdx.x == 0) {
        part_r[(i64)b * gridDim.x + blockIdx.x] = a;
        part_v[(i64)b * gridDim.x + blockIdx.x] = c;
    }
}

// Pivot certainty of a factor: per column j (permuted order) the ratio of
// the pivot L_jj^2 to the assembled diagonal a_jj of H_gamma (FP64:
// H_jj + D_x,j + delta + gamma * sum_i J_ij^2). Cholesky's pivot is a_jj less
// the squares already eliminated from the row, so a small ratio means the
// pivot is what is left after cancellation, known to fewer bits of the
// factor's precision. Block maxima of -ratio (so that k_reduce_max gives
// -min) into part.
// the FP64 diagonal of H_gamma = H + D_x + delta I + gamma J^T J per
// (instance, permuted column), the quantity k_pivot_ratio divides by
__global__ __launch_bounds__(kBlock) void k_hg_diag(SymView S, ValView V, double* __restrict__ out) {
    const int b = blockIdx.y;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < S.n; i += (i64)gridDim.x * blockDim.x) {
        const int k = S.G > 1 ? S.xp_mem[i] : 0;
        const double* HF = V.HF + (i64)b * S.nnzHF;
        const double* JT = V.JT + (i64)b * S.nnzJ;
        double d = V.Dxp[(i64)b * S.n + i] + V.delta[(i64)b * S.G + k], jj = 0.0;
        for (i64 q = S.HF_rowptr[i]; q < S.HF_rowptr[i + 1]; q++)
            if (S.HF_col[q] == i) d += HF[q];
        for (i64 q = S.JT_rowptr[i]; q < S.JT_rowptr[i + 1]; q++) jj += JT[q] * JT[q];
        out[(i64)b * S.n + i] = d + V.gamma[(i64)b * S.G + k] * jj;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pivot_ratio(SymView S, ValView V, const T* __restrict__ Dinv,
                                                        double* __restrict__ part) {
    __shared__ double sh[kBlock / kWave];
    const int b = blockIdx.y;
    const Blk bk = blk_of(S.rblk, blockIdx.x);
    const i64 i = bk.lo + threadIdx.x;
    double a = -INFINITY;
    if (i < bk.hi && i < S.n) {
        const double* HF = V.HF + (i64)b * S.nnzHF;
        const double* JT = V.JT + (i64)b * S.nnzJ;
        double d = V.Dxp[(i64)b * S.n + i] + V.delta[(i64)b * S.G + bk.k], jj = 0.0;
        for (i64 k = S.HF_rowptr[i]; k < S.HF_rowptr[i + 1]; k++)
            if (S.HF_col[k] == i) d += HF[k];
        for (i64 k = S.JT_rowptr[i]; k < S.JT_rowptr[i + 1]; k++) jj += JT[k] * JT[k];
        d += V.gamma[(i64)b * S.G + bk.k] * jj;
        const double r = (double)Dinv[(i64)b * S.n + i];
        a = -1.0 / (r * r * d);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) a = fmax(a, __shfl_down(a, o, kWave));
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = -INFINITY;
        for (int t = 0; t < (int)(blockDim.x / kWave); t++) r = fmax(r, sh[t]);
        part[(i64)b * gridDim.x + blockIdx.x] = r;
    }
}

// block maxima of the row sums of |H + D_x + delta I| (rows of x, into
// part_h) and of |J| (rows of J, into part_j), for the gamma heuristic
__global__ __launch_bounds__(kBlock) void k_gamma_rows(SymView S, ValView V, double* __restrict__ part_h,
                                                       double* __restrict__ part_j) {
    __shared__ double sh[2][kBlock / kWave];
    const int b = blockIdx.y;
    const Blk bk = blk_of(S.rblk, blockIdx.x);
    const i64 i = bk.lo + threadIdx.x;
    double a = 0.0, c = 0.0;
    if (i < bk.hi && i < S.n) {
        const double* HF = V.HF + (i64)b * S.nnzHF;
        double dsum = V.Dxp[(i64)b * S.n + i] + V.delta[(i64)b * S.G + bk.k];
        for (i64 k = S.HF_rowptr[i]; k < S.HF_rowptr[i + 1]; k++) {
            if (S.HF_col[k] == i) dsum += HF[k];
            else a += fabs(HF[k]);
        }
        a += fabs(dsum);
    } else if (i < bk.hi) {
        const i64 r = i - S.n;
        const double* J = V.J + (i64)b * S.nnzJ;
        for (i64 k = S.J_rowptr[r]; k < S.J_rowptr[r + 1]; k++) c += fabs(J[k]);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        a = fmax(a, __shfl_down(a, o, kWave));
        c = fmax(c, __shfl_down(c, o, kWave));
    }
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) {
        sh[0][wid] = a;
        sh[1][wid] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ra = 0.0, rc = 0.0;
        for (int t = 0; t < (int)(blockDim.x / kWave); t++) {
            ra = fmax(ra, sh[0][t]);
            rc = fmax(rc, sh[1][t]);
        }
        part_h[(i64)b * gridDim.x + blockIdx.x] = ra;
        part_j[(i64)b * gridDim.x + blockIdx.x] = rc;
    }
}

// out[b * G + k] = max of the partials of member k (grid (nb, G))
__global__ void k_reduce_max(const double* part, int nblk, const i32* off, double* out, double init) {
    const int b = blockIdx.x, k = blockIdx.y;
    if (threadIdx.x == 0) {
        double r = init;
        for (int i = off[k]; i < off[k + 1]; i++) r = fmax(r, part[(i64)b * nblk + i]);
        out[(i64)b * gridDim.y + k] = r;
    }
}

}  // namespace hkkt
