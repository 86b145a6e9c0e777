// The n x n steps of near-separable NMF on the GPU, in FP64: extreme-column
// selection (SPA, greedy XRAY, Gaussian-projection selection), the NNLS solve
// for H and the relative residual.  The paper notes that these run on O(n^2)
// data and are cheap even in serial (Sec. 2.4); they are single-workgroup or
// one-thread-per-column kernels, stream-ordered, with no host synchronisation.
#include <float.h>

#include "common.hpp"

namespace tsnmf {

namespace {

constexpr int kThreads = 256;

// Block-wide argmax over (value, index) pairs; ties go to the smaller index.
// Every thread gets the result.  `sv`/`si` are LDS scratch of kThreads entries.
__device__ void block_argmax(double v, int idx, double* sv, int* si, double* out_v, int* out_i) {
    const int t = threadIdx.x;
    sv[t] = v;
    si[t] = idx;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
            const double ov = sv[t + s];
            const int oi = si[t + s];
            if (ov > sv[t] || (ov == sv[t] && oi < si[t])) {
                sv[t] = ov;
                si[t] = oi;
            }
        }
        __syncthreads();
    }
    *out_v = sv[0];
    *out_i = si[0];
    __syncthreads();
}

__device__ double block_sum(double v, double* sv) {
    const int t = threadIdx.x;
    sv[t] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s) sv[t] += sv[t + s];
        __syncthreads();
    }
    const double r = sv[0];
    __syncthreads();
    return r;
}

// ---- SPA (Sec. 2.1) -------------------------------------------------------------
// Z (p x n, row-major in the workspace) starts as M diag(1/colscale); each pick
// j* = argmax_j ||Z(:, j)||^2 over unpicked columns, then Z <- Z - u (u^T Z)
// with u = Z(:, j*) / ||Z(:, j*)||.  Thread j owns column j (n <= 256); the
// rows may be as many as the projection's k (p <= kSpaMaxRows), so that SPA
// also runs on (G^T X) D^{-1} (Sec. 2.3, Sec. 3.3).
constexpr int kSpaMaxRows = 4096;
__global__ void __launch_bounds__(kThreads) spa_kernel(const double* __restrict__ M, int p, int n, int ldm,
                                                       const double* __restrict__ colscale, int r, int* K,
                                                       double* score, int* info, double* Z) {
    __shared__ double sv[kThreads];
    __shared__ int si[kThreads];
    __shared__ double u[kSpaMaxRows];
    const int j = threadIdx.x;
    const bool col = j < n;
    const double sc = (col && colscale != nullptr) ? 1.0 / colscale[j] : 1.0;
    if (col)
        for (int i = 0; i < p; ++i) Z[(int64_t)i * n + j] = M[(int64_t)j * ldm + i] * sc;
    bool chosen = false;
    int picked = 0;
    for (int t = 0; t < r; ++t) {
        double s = 0.0;
        if (col)
            for (int i = 0; i < p; ++i) {
                const double z = Z[(int64_t)i * n + j];
                s = __builtin_fma(z, z, s);
            }
        double best;
        int bj;
        block_argmax((col && !chosen) ? s : -DBL_MAX, col ? j : 0x7fffffff, sv, si, &best, &bj);
        if (!(best > 0.0)) break;
        picked = t + 1;
        if (j == 0) {
            K[t] = bj;
            if (score != nullptr) score[t] = best;
        }
        if (j == bj) chosen = true;
        const double inv = 1.0 / __builtin_sqrt(best);
        for (int i = j; i < p; i += kThreads) u[i] = Z[(int64_t)i * n + bj] * inv;
        __syncthreads();
        if (col) {
            double w = 0.0;
            for (int i = 0; i < p; ++i) w = __builtin_fma(u[i], Z[(int64_t)i * n + j], w);
            for (int i = 0; i < p; ++i) Z[(int64_t)i * n + j] -= u[i] * w;
        }
        __syncthreads();
    }
    if (j == 0) {
        *info = picked;
        for (int t = picked; t < r; ++t) {
            K[t] = -1;
            if (score != nullptr) score[t] = 0.0;
        }
    }
}

// ---- Gaussian-projection selection (Sec. 2.3) -------------------------------------
// For each row l of Y diag(1/colscale) (FP64 quotients, as exact IEEE
// divisions): argmin and argmax (ties -> smallest index) are counted; columns
// are ranked by count (descending), then index.
__global__ void __launch_bounds__(kThreads) gp_select_kernel(const float* __restrict__ Y, int k, int n, int ldy,
                                                             const double* __restrict__ colscale, int r, int* K,
                                                             int* counts_out, int* info) {
    __shared__ int cnt[256];
    const int t = threadIdx.x;
    if (t < n) cnt[t] = 0;
    __syncthreads();
    for (int l = t; l < k; l += kThreads) {
        double mn = 0.0, mx = 0.0;
        int imn = 0, imx = 0;
        for (int j = 0; j < n; ++j) {
            double v = (double)Y[(int64_t)j * ldy + l];
            if (colscale != nullptr) v = v / colscale[j];
            if (j == 0 || v < mn) { mn = v; imn = j; }
            if (j == 0 || v > mx) { mx = v; imx = j; }
        }
        atomicAdd(&cnt[imn], 1);
        atomicAdd(&cnt[imx], 1);
    }
    __syncthreads();
    if (t < n) {
        const int c = cnt[t];
        if (counts_out != nullptr) counts_out[t] = c;
        int rank = 0, nz = 0;
        for (int j = 0; j < n; ++j) {
            const int cj = cnt[j];
            nz += cj > 0;
            rank += (cj > c) || (cj == c && j < t);
        }
        if (c > 0 && rank < r) K[rank] = t;
        if (t == 0) {
            const int got = nz < r ? nz : r;
            *info = got;
            for (int q = got; q < r; ++q) K[q] = -1;
        }
    }
}

// ---- NNLS (Sec. 2.4) ----------------------------------------------------------------
// Stage 1 (one workgroup): Householder QR of A = M(:, K) (p x r), applied to
// all columns of M: the top r rows give R_A (r x r) and C = Q_A^T M.  Then
// min_{y >= 0} ||A y - M(:, i)|| has the same minimiser as
// min_{y >= 0} ||R_A y - C(:, i)|| (Q_A is orthogonal), with the same
// gradient A^T (b - A y) = R_A^T (c - R_A y).
// Stage 2 (one thread per column): Lawson-Hanson on the r x r problem, the
// unconstrained subproblems solved by Householder QR of R_A(:, P).

struct NnlsWork {
    double* aug;      // p x (r + n) column-major: [A | M]
    double* RA;       // r x r column-major
    double* C;        // r x n column-major
    double* anorm1;   // ||A||_1; the next slot is 1.0 when K holds an index outside [0, n)
    double* scratch;  // per column: r * r + 6 r doubles
    const int* skip;  // when non-null and nonzero, do nothing (XRAY after an early stop)
};

// 1 when some K[q] (q < r) is outside [0, n).  Checked before any access that
// uses K, so a bad index never reaches memory.
__device__ int bad_indices(const int* K, int r, int n) {
    int bad = 0;
    for (int q = 0; q < r; ++q) bad |= (K[q] < 0 || K[q] >= n);
    return bad;
}

__global__ void __launch_bounds__(kThreads) nnls_qr_kernel(const double* __restrict__ M, int p, int n, int ldm,
                                                           const int* __restrict__ K, int r, NnlsWork w) {
    __shared__ double sv[kThreads];
    __shared__ double v[256];
    __shared__ int badk;
    const int t = threadIdx.x;
    if (w.skip != nullptr && w.skip[0] != 0) return;
    if (t == 0) {
        badk = bad_indices(K, r, n);
        w.anorm1[1] = badk ? 1.0 : 0.0;
    }
    __syncthreads();
    if (badk) return;
    const int ncol = r + n;
    double* aug = w.aug;
    for (int c = t; c < ncol; c += kThreads) {
        const int src = c < r ? K[c] : c - r;
        for (int i = 0; i < p; ++i) aug[(int64_t)c * p + i] = M[(int64_t)src * ldm + i];
    }
    // ||A||_1 = largest column l1 norm of A
    double a1 = 0.0;
    for (int c = t; c < r; c += kThreads) {
        double s = 0.0;
        for (int i = 0; i < p; ++i) s += __builtin_fabs(aug[(int64_t)c * p + i]);
        a1 = s > a1 ? s : a1;
    }
    sv[t] = a1;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s) sv[t] = sv[t] > sv[t + s] ? sv[t] : sv[t + s];
        __syncthreads();
    }
    if (t == 0) *w.anorm1 = sv[0];
    __syncthreads();
    for (int j = 0; j < r && j < p; ++j) {
        double* col = aug + (int64_t)j * p;
        double part = 0.0;
        for (int i = j + 1 + t; i < p; i += kThreads) part = __builtin_fma(col[i], col[i], part);
        const double sigma = block_sum(part, sv);
        const double alpha = col[j];
        double beta = alpha, tau = 0.0, sc = 0.0;
        if (sigma != 0.0) {
            const double nrm = __builtin_sqrt(alpha * alpha + sigma);
            beta = alpha >= 0.0 ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            sc = 1.0 / (alpha - beta);
        }
        for (int i = j + t; i < p; i += kThreads) v[i] = (i == j) ? 1.0 : col[i] * sc;
        __syncthreads();
        for (int c = j + 1 + t; c < ncol; c += kThreads) {
            double* cc = aug + (int64_t)c * p;
            double d = 0.0;
            for (int i = j; i < p; ++i) d = __builtin_fma(v[i], cc[i], d);
            d *= tau;
            for (int i = j; i < p; ++i) cc[i] -= d * v[i];
        }
        __syncthreads();
        if (t == 0) col[j] = beta;
        for (int i = j + 1 + t; i < p; i += kThreads) col[i] = 0.0;
        __syncthreads();
    }
    // R_A (rows beyond p stay zero) and C
    for (int c = t; c < r; c += kThreads)
        for (int i = 0; i < r; ++i) w.RA[(int64_t)c * r + i] = (i <= c && i < p) ? aug[(int64_t)c * p + i] : 0.0;
    for (int c = t; c < n; c += kThreads)
        for (int i = 0; i < r; ++i) w.C[(int64_t)c * r + i] = i < p ? aug[(int64_t)(r + c) * p + i] : 0.0;
}

// Least squares min ||B s - c|| for the columns of R_A listed in idx[0..q-1]
// (Householder QR in `a` (r x q) and `rhs` (r)); writes s into sol[idx[.]].
__device__ void ls_passive(const double* RA, int r, const double* c, const int* idx, int q, double* a, double* rhs,
                           double* sol) {
    for (int jj = 0; jj < q; ++jj)
        for (int i = 0; i < r; ++i) a[jj * r + i] = RA[(int64_t)idx[jj] * r + i];
    for (int i = 0; i < r; ++i) rhs[i] = c[i];
    for (int j = 0; j < q; ++j) {
        double sigma = 0.0;
        for (int i = j + 1; i < r; ++i) sigma += a[j * r + i] * a[j * r + i];
        const double alpha = a[j * r + j];
        if (sigma == 0.0) continue;
        const double nrm = __builtin_sqrt(alpha * alpha + sigma);
        const double beta = alpha >= 0.0 ? -nrm : nrm;
        const double tau = (beta - alpha) / beta;
        const double sc = 1.0 / (alpha - beta);
        for (int i = j + 1; i < r; ++i) a[j * r + i] *= sc;     // v = [1; a(j+1:, j)]
        for (int cc = j + 1; cc < q; ++cc) {
            double d = a[cc * r + j];
            for (int i = j + 1; i < r; ++i) d += a[j * r + i] * a[cc * r + i];
            d *= tau;
            a[cc * r + j] -= d;
            for (int i = j + 1; i < r; ++i) a[cc * r + i] -= d * a[j * r + i];
        }
        double d = rhs[j];
        for (int i = j + 1; i < r; ++i) d += a[j * r + i] * rhs[i];
        d *= tau;
        rhs[j] -= d;
        for (int i = j + 1; i < r; ++i) rhs[i] -= d * a[j * r + i];
        a[j * r + j] = beta;
    }
    for (int j = q - 1; j >= 0; --j) {
        double s = rhs[j];
        for (int cc = j + 1; cc < q; ++cc) s -= a[cc * r + j] * sol[idx[cc]];
        sol[idx[j]] = s / a[j * r + j];
    }
}

__global__ void __launch_bounds__(64) nnls_solve_kernel(const double* __restrict__ M, int p, int n, int ldm,
                                                        const int* __restrict__ K, int r, NnlsWork w, double* H,
                                                        int ldh, double* resid2, int* info) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (w.skip != nullptr && w.skip[0] != 0) return;
    if (w.anorm1[1] != 0.0) {                  // invalid K: no solve, NaN results
        for (int q = 0; q < r; ++q) H[(int64_t)i * ldh + q] = __builtin_nan("");
        if (resid2 != nullptr) resid2[i] = __builtin_nan("");
        if (info != nullptr) info[i] = 2;
        return;
    }
    const double* RA = w.RA;
    const double* c = w.C + (int64_t)i * r;
    double* x = w.scratch + (int64_t)i * (r * r + 6 * r);
    double* s = x + r;
    double* g = s + r;
    double* pass = g + r;          // 1.0 when in the passive set
    int* idx = (int*)(pass + r);   // passive indices (r ints fit in r doubles)
    double* rhs = pass + 2 * r;
    double* a = rhs + r;
    const int maxit = 3 * r;
    const double tol = 10.0 * DBL_EPSILON * (*w.anorm1) * (double)(p > r ? p : r);
    for (int q = 0; q < r; ++q) { x[q] = 0.0; pass[q] = 0.0; }
    int inf = 0, outer = 0;
    while (true) {
        // g = R_A^T (c - R_A x)
        for (int q = 0; q < r; ++q) {
            double e = c[q];
            for (int u = q; u < r; ++u) e -= RA[(int64_t)u * r + q] * x[u];
            s[q] = e;                                  // residual, reused below
        }
        for (int q = 0; q < r; ++q) {
            double d = 0.0;
            for (int u = 0; u <= q; ++u) d += RA[(int64_t)q * r + u] * s[u];
            g[q] = d;
        }
        int tbest = -1;
        double gbest = -DBL_MAX;
        for (int q = 0; q < r; ++q)
            if (pass[q] == 0.0 && g[q] > gbest) { gbest = g[q]; tbest = q; }
        if (tbest < 0 || !(gbest > tol)) break;
        if (outer >= maxit) { inf = 1; break; }
        ++outer;
        pass[tbest] = 1.0;
        int inner = 0;
        while (true) {
            int qn = 0;
            for (int q = 0; q < r; ++q)
                if (pass[q] != 0.0) idx[qn++] = q;
            for (int q = 0; q < r; ++q) s[q] = 0.0;
            ls_passive(RA, r, c, idx, qn, a, rhs, s);
            bool allpos = true;
            for (int q = 0; q < qn; ++q) allpos = allpos && s[idx[q]] > 0.0;
            if (allpos) {
                for (int q = 0; q < r; ++q) x[q] = s[q];
                break;
            }
            // Largest step keeping x >= 0 over the indices with s <= 0.  An
            // index already at zero (x = 0) allows no step: its ratio is 0,
            // not 0 / 0.  The index that limits the step is set to zero and
            // leaves P, so this loop ends within qn rounds.
            double alpha = DBL_MAX;
            int ubest = -1;
            for (int q = 0; q < qn; ++q) {
                const int u = idx[q];
                if (s[u] <= 0.0) {
                    const double al = x[u] > 0.0 ? x[u] / (x[u] - s[u]) : 0.0;
                    if (al < alpha) { alpha = al; ubest = u; }
                }
            }
            if (ubest < 0) {                 // no finite step (NaN in the subproblem)
                inf = 1;
                break;
            }
            for (int q = 0; q < r; ++q) x[q] += alpha * (s[q] - x[q]);
            x[ubest] = 0.0;
            int left = 0;
            for (int q = 0; q < r; ++q) {
                if (pass[q] != 0.0 && x[q] <= tol) { pass[q] = 0.0; x[q] = 0.0; }
                left += pass[q] != 0.0;
            }
            if (left == 0 || ++inner > r) break;
        }
    }
    for (int q = 0; q < r; ++q) H[(int64_t)i * ldh + q] = x[q];
    if (resid2 != nullptr) {
        double e2 = 0.0;
        for (int row = 0; row < p; ++row) {
            double e = -M[(int64_t)i * ldm + row];
            for (int q = 0; q < r; ++q) e += M[(int64_t)K[q] * ldm + row] * x[q];
            e2 += e * e;
        }
        resid2[i] = e2;
    }
    if (info != nullptr) info[i] = inf;
}

// ---- residual (Sec. 4) --------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) residual_kernel(const double* __restrict__ M, int p, int n, int ldm,
                                                            const int* __restrict__ K, int r,
                                                            const double* __restrict__ H, int ldh, double* out) {
    __shared__ double sv[kThreads];
    if (bad_indices(K, r, n)) {
        if (threadIdx.x == 0) *out = __builtin_nan("");
        return;
    }
    double e2 = 0.0, m2 = 0.0;
    for (int j = threadIdx.x; j < n; j += kThreads) {
        for (int i = 0; i < p; ++i) {
            const double mij = M[(int64_t)j * ldm + i];
            double e = mij;
            for (int q = 0; q < r; ++q) e -= M[(int64_t)K[q] * ldm + i] * H[(int64_t)j * ldh + q];
            e2 += e * e;
            m2 += mij * mij;
        }
    }
    const double E = block_sum(e2, sv);
    const double T = block_sum(m2, sv);
    if (threadIdx.x == 0) *out = T > 0.0 ? E / T : 0.0;
}

// ---- greedy XRAY (Sec. 2.1) -------------------------------------------------------
// One pick: score_j = ||Res^T M(:, j)|| / ||M(:, j)|| over unpicked columns with
// ||M(:, j)|| > 0 (Res = M before the first pick), argmax, append to K.
__global__ void __launch_bounds__(kThreads) xray_pick_kernel(const double* __restrict__ M, int p, int n, int ldm,
                                                             const double* __restrict__ Res, int t, int* K,
                                                             int* state) {
    __shared__ double sv[kThreads];
    __shared__ int si[kThreads];
    if (state[0] != 0) return;                       // stopped earlier
    const int j = threadIdx.x;
    double score = -DBL_MAX;
    if (j < n) {
        bool used = false;
        for (int q = 0; q < t; ++q) used = used || K[q] == j;
        double mn = 0.0;
        for (int i = 0; i < p; ++i) mn += M[(int64_t)j * ldm + i] * M[(int64_t)j * ldm + i];
        if (!used && mn > 0.0) {
            double s2 = 0.0;
            for (int c = 0; c < n; ++c) {
                double d = 0.0;
                for (int i = 0; i < p; ++i) d += Res[(int64_t)c * p + i] * M[(int64_t)j * ldm + i];
                s2 += d * d;
            }
            score = __builtin_sqrt(s2) / __builtin_sqrt(mn);
        }
    }
    double best;
    int bj;
    block_argmax(score, j < n ? j : 0x7fffffff, sv, si, &best, &bj);
    if (j == 0) {
        if (best == -DBL_MAX) {
            state[0] = 1;                            // nothing left to pick
        } else {
            K[t] = bj;
            state[1] = t + 1;
        }
    }
}

// Res = M - M(:, K[0..t]) H  (p x n, column-major, ld p)
__global__ void xray_residual_kernel(const double* __restrict__ M, int p, int n, int ldm, const int* __restrict__ K,
                                     int t, const double* __restrict__ H, int ldh, double* Res,
                                     const int* state) {
    if (state[0] != 0) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)p * n) return;
    const int i = (int)(e % p), j = (int)(e / p);
    double v = M[(int64_t)j * ldm + i];
    for (int q = 0; q < t; ++q) v -= M[(int64_t)K[q] * ldm + i] * H[(int64_t)j * ldh + q];
    Res[e] = v;
}

__global__ void copy_matrix_kernel(const double* __restrict__ M, int p, int n, int ldm, double* Res) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)p * n) return;
    Res[e] = M[(e / p) * ldm + e % p];
}

__global__ void xray_finish_kernel(int r, int* K, int* info, const int* state) {
    if (threadIdx.x == 0) {
        const int got = state[1];
        *info = got;
        for (int q = got; q < r; ++q) K[q] = -1;
    }
}

__global__ void zero_ints_kernel(int* p, int count) {
    if ((int)threadIdx.x < count) p[threadIdx.x] = 0;
}

size_t nnls_bytes(int p, int n, int r) {
    return ((size_t)p * (r + n) + (size_t)r * r + (size_t)r * n + 2 + (size_t)n * (r * r + 6 * r)) * 8 + 1024;
}

NnlsWork nnls_layout(void* base, int p, int n, int r) {
    NnlsWork w{};
    double* d = (double*)base;
    w.aug = d;
    d += (size_t)p * (r + n);
    w.RA = d;
    d += (size_t)r * r;
    w.C = d;
    d += (size_t)r * n;
    w.anorm1 = d;
    d += 2;
    w.scratch = d;
    return w;
}

int nnls_launch(const double* M, int p, int n, int ldm, const int* K, int r, double* H, int ldh, double* resid2,
                int* info, void* ws, hipStream_t stream, const int* skip = nullptr) {
    NnlsWork w = nnls_layout(ws, p, n, r);
    w.skip = skip;
    hipLaunchKernelGGL(nnls_qr_kernel, dim3(1), dim3(kThreads), 0, stream, M, p, n, ldm, K, r, w);
    TSNMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(nnls_solve_kernel, dim3((n + 63) / 64), dim3(64), 0, stream, M, p, n, ldm, K, r, w, H, ldh,
                       resid2, info);
    TSNMF_LAUNCH_CHECK();
    return TSNMF_OK;
}

}  // namespace

int select_spa_impl(const double* M, int p, int n, int ldm, const double* colscale, int r, int* K, double* score,
                    int* info, hipStream_t stream) {
    void* ws = nullptr;
    if (int st = workspace_get(kTicketBytes + (size_t)p * n * 8, stream, &ws)) return st;
    hipLaunchKernelGGL(spa_kernel, dim3(1), dim3(kThreads), 0, stream, M, p, n, ldm, colscale, r, K, score, info,
                       (double*)((char*)ws + kTicketBytes));
    TSNMF_LAUNCH_CHECK();
    return TSNMF_OK;
}

int select_gp_impl(const float* Y, int k, int n, int ldy, const double* colscale, int r, int* K, int* counts,
                   int* info, hipStream_t stream) {
    hipLaunchKernelGGL(gp_select_kernel, dim3(1), dim3(kThreads), 0, stream, Y, k, n, ldy, colscale, r, K, counts,
                       info);
    TSNMF_LAUNCH_CHECK();
    return TSNMF_OK;
}

int nnls_impl(const double* M, int p, int n, int ldm, const int* K, int r, double* H, int ldh, double* resid2,
              int* info, hipStream_t stream) {
    void* ws = nullptr;
    if (int st = workspace_get(kTicketBytes + nnls_bytes(p, n, r), stream, &ws)) return st;
    return nnls_launch(M, p, n, ldm, K, r, H, ldh, resid2, info, (char*)ws + kTicketBytes, stream);
}

int residual_impl(const double* M, int p, int n, int ldm, const int* K, int r, const double* H, int ldh,
                  double* relerr, hipStream_t stream) {
    hipLaunchKernelGGL(residual_kernel, dim3(1), dim3(kThreads), 0, stream, M, p, n, ldm, K, r, H, ldh, relerr);
    TSNMF_LAUNCH_CHECK();
    return TSNMF_OK;
}

int select_xray_impl(const double* M, int p, int n, int ldm, int r, int* K, int* info, hipStream_t stream) {
    // workspace: state (2 ints), Res (p x n), H (r x n), NNLS work
    const size_t res_b = (size_t)p * n * 8, h_b = (size_t)r * n * 8;
    void* ws = nullptr;
    if (int st = workspace_get(kTicketBytes + 256 + res_b + h_b + nnls_bytes(p, n, r), stream, &ws)) return st;
    char* b = (char*)ws + kTicketBytes;
    int* state = (int*)b;
    double* Res = (double*)(b + 256);
    double* H = (double*)(b + 256 + res_b);
    void* nw = b + 256 + res_b + h_b;
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, stream, state, 2);
    TSNMF_LAUNCH_CHECK();
    const int64_t pn = (int64_t)p * n;
    hipLaunchKernelGGL(copy_matrix_kernel, dim3((unsigned)((pn + 255) / 256)), dim3(256), 0, stream, M, p, n, ldm,
                       Res);
    TSNMF_LAUNCH_CHECK();
    for (int t = 0; t < r && t < n; ++t) {
        hipLaunchKernelGGL(xray_pick_kernel, dim3(1), dim3(kThreads), 0, stream, M, p, n, ldm, Res, t, K, state);
        TSNMF_LAUNCH_CHECK();
        if (t + 1 == r) break;
        // H = NNLS(M(:, K[0..t]), M) and the new residual; both do nothing on the
        // device once no column was left to pick (K[t] is then unset)
        if (int st = nnls_launch(M, p, n, ldm, K, t + 1, H, t + 1, nullptr, nullptr, nw, stream, state)) return st;
        hipLaunchKernelGGL(xray_residual_kernel, dim3((unsigned)((pn + 255) / 256)), dim3(256), 0, stream, M, p, n,
                           ldm, K, t + 1, H, t + 1, Res, state);
        TSNMF_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(xray_finish_kernel, dim3(1), dim3(64), 0, stream, r, K, info, state);
    TSNMF_LAUNCH_CHECK();
    return TSNMF_OK;
}

}  // namespace tsnmf
