// The n x n steps of near-separable NMF on the GPU, in FP64: extreme-column
// selection (SPA, greedy XRAY, Gaussian-projection selection), the NNLS solve
// for H, the relative residual and its curve over ranks.  The paper notes that
// these run on O(n^2) data and are cheap even in serial (Sec. 2.4); they are
// single-workgroup kernels (the matrices in LDS when they fit) or one wave per
// column of H, stream-ordered, with no host synchronisation.
#include <float.h>

#include "common.hpp"
#include "wave.hpp"

namespace tsnmf {

namespace {

constexpr int kThreads = 256;

// v as held by lane `src` (wave-uniform).
__device__ __forceinline__ double lane_value(double v, int src) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One 64-lane wave: the sum of v over the lanes by the permlane and DPP
// stages (partners L ^ 32, 16, 15, 7, 2, 1: every stage adds a disjoint set of
// lanes, and partners add the same two values), taken from lane 0 so that it
// is wave-uniform by construction.
__device__ __forceinline__ double wave_sum(double v) {
    v = allreduce_stage<5>(v);
    v = allreduce_stage<4>(v);
    v = allreduce_stage<3>(v);
    v = allreduce_stage<2>(v);
    v = allreduce_stage<1>(v);
    v = allreduce_stage<0>(v);
    return lane_value(v, 0);
}

// The value of lane L ^ m at the stage on lane bit BIT (m as in wave_sum).
template <int BIT> __device__ __forceinline__ uint32_t partner_u32(uint32_t x) {
    if constexpr (BIT == 5) {
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return (threadIdx.x & 32) ? r[0] : r[1];
    } else if constexpr (BIT == 4) {
        const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        return (threadIdx.x & 16) ? r[0] : r[1];
    } else {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DppCtrl<BIT>::v, 0xf, 0xf, false);
    }
}

template <int BIT> __device__ __forceinline__ void argmax_stage(double& v, int& idx) {
    const double ov = mk64(partner_u32<BIT>(hi32(v)), partner_u32<BIT>(lo32(v)));
    const int oi = (int)partner_u32<BIT>((uint32_t)idx);
    if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
    }
}

// The (value, index) pair with the larger value, ties to the smaller index,
// over the wave; lane 0's result is the one returned to every lane.
__device__ __forceinline__ void wave_argmax_pair(double& v, int& idx) {
    argmax_stage<5>(v, idx);
    argmax_stage<4>(v, idx);
    argmax_stage<3>(v, idx);
    argmax_stage<2>(v, idx);
    argmax_stage<1>(v, idx);
    argmax_stage<0>(v, idx);
    v = lane_value(v, 0);
    idx = __builtin_amdgcn_readfirstlane(idx);
}

// Index of the largest v over the wave, ties to the smaller index; lanes
// without a candidate pass (-inf, 64), so 64 means none.
__device__ __forceinline__ int wave_argmax(double v, int idx) {
    wave_argmax_pair(v, idx);
    return idx;
}

// Block-wide argmax over (value, index) pairs; ties go to the smaller index.
// Every thread gets the result: each wave reduces by shuffles, then every
// thread combines the waves' pairs in wave order (the winner is the same in
// any order: larger value, then smaller index).  `sv`/`si` are LDS scratch of
// at least kThreads / 64 entries.
__device__ void block_argmax(double v, int idx, double* sv, int* si, double* out_v, int* out_i) {
    wave_argmax_pair(v, idx);
    if ((threadIdx.x & 63) == 0) {
        sv[threadIdx.x >> 6] = v;
        si[threadIdx.x >> 6] = idx;
    }
    __syncthreads();
    v = sv[0];
    idx = si[0];
    for (int w = 1; w < kThreads / 64; ++w) {
        const double ov = sv[w];
        const int oi = si[w];
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
    *out_v = v;
    *out_i = idx;
    __syncthreads();
}

// Block-wide sum: per wave by shuffles, then the waves' sums in wave order.
__device__ double block_sum(double v, double* sv) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sv[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sv[0];
    for (int w = 1; w < kThreads / 64; ++w) r += sv[w];
    __syncthreads();
    return r;
}

// ---- SPA (Sec. 2.1) -------------------------------------------------------------
// Z (p x n, row-major in the workspace) starts as M diag(1/colscale); each pick
// j* = argmax_j ||Z(:, j)||^2 over unpicked columns, then Z <- Z - u (u^T Z)
// with u = Z(:, j*) / ||Z(:, j*)||.  Thread j owns column j (n <= 256); the
// rows may be as many as the projection's k (p <= kSpaMaxRows), so that SPA
// also runs on (G^T X) D^{-1} (Sec. 2.3, Sec. 3.3).
// With ZL, Z lives in LDS after u (p (n + 1) doubles), else in `Zg`.
constexpr int kSpaMaxRows = 4096;
constexpr size_t kLdsCap = 150 * 1024;   // dynamic LDS these kernels may take
__host__ __device__ constexpr bool spa_z_in_lds(int p, int n) {
    return (size_t)p * (n + 1) * sizeof(double) <= kLdsCap;
}
template <bool ZL>
__global__ void __launch_bounds__(kThreads) spa_kernel(const double* __restrict__ M, int p, int n, int ldm,
                                                       const double* __restrict__ colscale, int r, int* K,
                                                       double* score, int* info, double* Zg) {
    extern __shared__ double spa_lds[];
    __shared__ double sv[kThreads / 64];
    __shared__ int si[kThreads / 64];
    double* u = spa_lds;
    double* Z = ZL ? spa_lds + p : Zg;
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
#pragma unroll 4
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
#pragma unroll 4
            for (int i = 0; i < p; ++i) w = __builtin_fma(u[i], Z[(int64_t)i * n + j], w);
#pragma unroll 4
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
// Stage 2 (one wave per column): Lawson-Hanson on the r x r problem, the
// unconstrained subproblems solved by Householder QR of R_A(:, P).

struct NnlsWork {
    double* aug;      // p x (r + n) column-major: [A | M]
    double* RA;       // r x r column-major
    double* C;        // r x n column-major
    double* anorm1;   // [0] ||A||_1, [1] 1.0 when K holds an index outside [0, n),
                      // [2] (prefix mode) the number of leading valid indices,
                      // then the l1 norm of every column of A
    const int* skip;  // when non-null and nonzero, do nothing (XRAY after an early stop)
    int prefix;       // factor the leading valid columns only (the rank sweep: every
                      // prefix K[0..r) shares the first r Householder steps)
};

// 1 when some K[q] (q < r) is outside [0, n).  Checked before any access that
// uses K, so a bad index never reaches memory.
__device__ int bad_indices(const int* K, int r, int n) {
    int bad = 0;
    for (int q = 0; q < r; ++q) bad |= (K[q] < 0 || K[q] >= n);
    return bad;
}

// With AL, [A | M] lives in LDS with an odd leading dimension (conflict-free
// column walks by consecutive threads), else in the workspace with ld p.
__host__ __device__ constexpr int nnls_qr_ld(int p, bool al) { return al ? (p | 1) : p; }
__host__ __device__ constexpr bool nnls_aug_in_lds(int p, int n, int r) {
    return (size_t)nnls_qr_ld(p, true) * (r + n) * sizeof(double) <= kLdsCap;
}
template <bool AL, int NT>
__global__ void __launch_bounds__(NT) nnls_qr_kernel(const double* __restrict__ M, int p, int n, int ldm,
                                                           const int* __restrict__ K, int r, NnlsWork w) {
    extern __shared__ double qr_lds[];
    __shared__ double sv[kThreads];
    __shared__ double v[256];
    __shared__ int badk, rvs;
    const int t = threadIdx.x;
    const int lda = nnls_qr_ld(p, AL);
    if (w.skip != nullptr && w.skip[0] != 0) return;
    if (t == 0) {
        if (w.prefix) {
            int rv = 0;
            while (rv < r && K[rv] >= 0 && K[rv] < n) ++rv;
            badk = 0;
            rvs = rv;
            w.anorm1[2] = (double)rv;
        } else {
            badk = bad_indices(K, r, n);
            rvs = r;
        }
        w.anorm1[1] = badk ? 1.0 : 0.0;
    }
    __syncthreads();
    if (badk) return;
    const int rv = rvs;                      // columns of A taken from M; the rest are zero
    const int ncol = r + n;
    double* aug = AL ? qr_lds : w.aug;
    double* cn1 = w.anorm1 + 3;
    for (int c = t; c < ncol; c += NT) {
        const int src = c < r ? (c < rv ? K[c] : -1) : c - r;
        for (int i = 0; i < p; ++i) aug[(int64_t)c * lda + i] = src >= 0 ? M[(int64_t)src * ldm + i] : 0.0;
    }
    // ||A||_1 = largest column l1 norm of A (each column's kept for the prefixes)
    double a1 = 0.0;
    for (int c = t; c < r; c += NT) {
        double s = 0.0;
        for (int i = 0; i < p; ++i) s += __builtin_fabs(aug[(int64_t)c * lda + i]);
        cn1[c] = s;
        a1 = s > a1 ? s : a1;
    }
    sv[t] = a1;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s) sv[t] = sv[t] > sv[t + s] ? sv[t] : sv[t + s];
        __syncthreads();
    }
    if (t == 0) *w.anorm1 = sv[0];
    __syncthreads();
    for (int j = 0; j < rv && j < p; ++j) {
        double* col = aug + (int64_t)j * lda;
        double part = 0.0;
        for (int i = j + 1 + t; i < p; i += NT) part = __builtin_fma(col[i], col[i], part);
        const double sigma = NT == 64 ? wave_sum(part) : block_sum(part, sv);
        const double alpha = col[j];
        double beta = alpha, tau = 0.0, sc = 0.0;
        if (sigma != 0.0) {
            const double nrm = __builtin_sqrt(alpha * alpha + sigma);
            beta = alpha >= 0.0 ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            sc = 1.0 / (alpha - beta);
        }
        for (int i = j + t; i < p; i += NT) v[i] = (i == j) ? 1.0 : col[i] * sc;
        __syncthreads();
        for (int c = j + 1 + t; c < ncol; c += NT) {
            double* cc = aug + (int64_t)c * lda;
            double d = 0.0;
#pragma unroll 4
            for (int i = j; i < p; ++i) d = __builtin_fma(v[i], cc[i], d);
            d *= tau;
#pragma unroll 4
            for (int i = j; i < p; ++i) cc[i] -= d * v[i];
        }
        __syncthreads();
        if (t == 0) col[j] = beta;
        for (int i = j + 1 + t; i < p; i += NT) col[i] = 0.0;
        __syncthreads();
    }
    // R_A (rows beyond p stay zero) and C
    for (int c = t; c < r; c += NT)
        for (int i = 0; i < r; ++i) w.RA[(int64_t)c * r + i] = (i <= c && i < p) ? aug[(int64_t)c * lda + i] : 0.0;
    for (int c = t; c < n; c += NT)
        for (int i = 0; i < r; ++i) w.C[(int64_t)c * r + i] = i < p ? aug[(int64_t)(r + c) * lda + i] : 0.0;
}

// Leading dimension of the LDS matrices of nnls_solve_kernel: odd, so that a
// lane-strided column walk of FP64 entries is free of bank conflicts.
__host__ __device__ constexpr int nnls_ld(int r) { return r | 1; }

__host__ __device__ constexpr size_t nnls_solve_lds(int r) {
    return ((size_t)(2 * r + 1) * nnls_ld(r) + 3 * 64 + 32) * sizeof(double);
}

// Stage 2: one wave per column i of M, lane q holding entry q of x, of the
// gradient, of the subproblem's solution and whether q is in the passive set
// (r <= 64).  R_A and the subproblem live in LDS.  The subproblem
// min ||R_A(:, P) s - c|| is factored by Householder steps on the passive
// columns with c appended as one more column, lane j' owning column j'.
// Column j of R_A(:, P) is R_A(:, P[j]), zero below row P[j]; the reflections
// of the earlier columns touch rows up to P[j'] < P[j] only, so it stays zero
// there and step j runs over rows j .. P[j] (the other terms are exact zeros).
// Column i of M: R_A is the leading r x r block of `RA` and c the first r
// entries of `ci` (column-major, leading dimension ldra); `lds` holds at least
// nnls_solve_lds(r) bytes.  Writes x to h (when non-null), ||M(:, K) x - M(:, i)||^2
// to *resid2 and the iteration-cap flag to *info (when non-null).
__device__ __forceinline__ void nnls_solve_wave(const double* __restrict__ M, int p, int ldm,
                                                const int* __restrict__ K, int r, int ldra,
                                                const double* __restrict__ RA, const double* __restrict__ ci,
                                                double tol, double* lds, int i, double* h, double* resid2,
                                                int* info) {
    const int L = (int)threadIdx.x;
    const bool lane_ok = L < r;
    const int ld = nnls_ld(r);
    double* sRA = lds;                        // R_A, column u at sRA + u ld
    double* sa = sRA + r * ld;                // subproblem: passive columns of R_A, then c
    double* sv = sa + (r + 1) * ld;           // Householder vector of the current step
    double* sx = sv + 64;                     // x, then c - R_A x, for the gradient
    double* se = sx + 64;
    int* sidx = (int*)(se + 64);              // passive indices, ascending
    for (int u = 0; u < r; ++u)
        if (lane_ok) sRA[u * ld + L] = RA[(int64_t)u * ldra + L];
    const double cq = lane_ok ? ci[L] : 0.0;
    const int maxit = 3 * r;
    const unsigned long long below = (1ull << L) - 1;   // lanes under this one
    double x = 0.0;
    bool pass = false;
    int inf = 0, outer = 0;
    __syncthreads();
    while (true) {
        // g = R_A^T (c - R_A x)
        sx[L] = x;
        __syncthreads();
        double e = cq;
#pragma unroll 4
        for (int u = 0; u < r; ++u)
            if (lane_ok && u >= L) e -= sRA[u * ld + L] * sx[u];
        se[L] = e;
        __syncthreads();
        double g = 0.0;
#pragma unroll 4
        for (int u = 0; u < r; ++u)
            if (lane_ok && u <= L) g += sRA[L * ld + u] * se[u];
        // entering index: the largest gradient outside P, when above tol
        const bool enter = lane_ok && !pass && g > tol;
        const int tbest = wave_argmax(enter ? g : -INFINITY, enter ? L : 64);
        if (tbest >= 64) break;
        if (outer >= maxit) {
            inf = 1;
            break;
        }
        ++outer;
        if (L == tbest) pass = true;
        int inner = 0;
        while (true) {
            const unsigned long long pm = __ballot(pass);
            const int qn = __popcll(pm);
            const int pos = __popcll(pm & below);      // this lane's place in P
            if (pass) sidx[pos] = L;
            __syncthreads();
            const int pj = sidx[L];                    // P[L] in lanes L < qn (read by every lane)
            for (int j = 0; j < qn; ++j) {
                const int src = __builtin_amdgcn_readlane(pj, j);
                if (lane_ok) sa[j * ld + L] = sRA[src * ld + L];
            }
            if (lane_ok) sa[qn * ld + L] = cq;
            __syncthreads();
            for (int j = 0; j < qn; ++j) {
                const int hi = __builtin_amdgcn_readlane(pj, j);   // last row that can be nonzero in column j
                if (hi == j) continue;                 // zero below the diagonal: sigma = 0, no step
                double* colj = sa + j * ld;
                const double aij = (L > j && L <= hi) ? colj[L] : 0.0;
                const double sigma = wave_sum(aij * aij);
                const double alpha = colj[j];
                if (sigma == 0.0) continue;            // wave-uniform
                const double nrm = __builtin_sqrt(alpha * alpha + sigma);
                const double beta = alpha >= 0.0 ? -nrm : nrm;
                const double tau = (beta - alpha) / beta;
                const double sc = 1.0 / (alpha - beta);
                if (L > j && L <= hi) {                // v = [1; a(j+1 .. hi, j) sc]
                    const double v = aij * sc;
                    colj[L] = v;
                    sv[L] = v;
                }
                __syncthreads();
                if (L > j && L <= qn) {                // the later columns and c
                    double* cc = sa + L * ld;
                    double d = cc[j];
#pragma unroll 4
                    for (int u = j + 1; u <= hi; ++u) d += sv[u] * cc[u];
                    d *= tau;
                    cc[j] -= d;
#pragma unroll 4
                    for (int u = j + 1; u <= hi; ++u) cc[u] -= d * sv[u];
                }
                if (L == j) colj[j] = beta;
                __syncthreads();
            }
            // back substitution, one column of the triangle per step
            // reciprocals of the diagonal formed together, off the serial chain
            const int Lq = L < qn ? L : 0;             // in-range index for every lane
            const double dinv = L < qn ? 1.0 / sa[Lq * ld + Lq] : 0.0;
            double acc = L < qn ? sa[qn * ld + Lq] : 0.0;
            double sol = 0.0;
            for (int c = qn - 1; c >= 0; --c) {
                const double sc = lane_value(acc, c) * lane_value(dinv, c);
                if (L == c) sol = sc;
                if (L < c) acc -= sa[c * ld + L] * sc;
            }
            const double sp = __shfl(sol, pos);        // solution entry of index L
            const double s = pass ? sp : 0.0;
            if (__ballot(pass && !(s > 0.0)) == 0) {  // all of P positive: accept
                x = s;
                break;
            }
            // Largest step keeping x >= 0 over the indices of P with s <= 0.  An
            // index already at zero (x = 0) allows no step: its ratio is 0,
            // not 0 / 0.  The index that limits the step is set to zero and
            // leaves P, so this loop ends within |P| rounds.
            const bool lim = pass && s <= 0.0;
            const double al = lim ? (x > 0.0 ? x / (x - s) : 0.0) : 0.0;
            const int ubest = wave_argmax(lim ? -al : -INFINITY, lim ? L : 64);
            if (ubest >= 64) {                         // no finite step (NaN in the subproblem)
                inf = 1;
                break;
            }
            const double step = lane_value(al, ubest);
            x += step * (s - x);
            if (L == ubest) x = 0.0;
            if (pass && x <= tol) {
                pass = false;
                x = 0.0;
            }
            const int left = __popcll(__ballot(pass));
            if (left == 0 || ++inner > r) break;
        }
    }
    if (lane_ok && h != nullptr) h[L] = x;
    if (resid2 != nullptr) {
        sv[L] = x;
        __syncthreads();
        double e2 = 0.0;
        for (int row = L; row < p; row += 64) {
            double e = -M[(int64_t)i * ldm + row];
            for (int q = 0; q < r; ++q) e += M[(int64_t)K[q] * ldm + row] * sv[q];
            e2 += e * e;
        }
        e2 = wave_sum(e2);
        if (L == 0) *resid2 = e2;
    }
    if (info != nullptr && L == 0) *info = inf;
}

__global__ void __launch_bounds__(64) nnls_solve_kernel(const double* __restrict__ M, int p, int n, int ldm,
                                                        const int* __restrict__ K, int r, NnlsWork w, double* H,
                                                        int ldh, double* resid2, int* info) {
    extern __shared__ double lds[];
    const int i = blockIdx.x;
    const int L = (int)threadIdx.x;
    if (w.skip != nullptr && w.skip[0] != 0) return;
    if (w.anorm1[1] != 0.0) {                  // invalid K: no solve, NaN results
        if (L < r) H[(int64_t)i * ldh + L] = __builtin_nan("");
        if (L == 0) {
            if (resid2 != nullptr) resid2[i] = __builtin_nan("");
            if (info != nullptr) info[i] = 2;
        }
        return;
    }
    const double tol = 10.0 * DBL_EPSILON * (*w.anorm1) * (double)(p > r ? p : r);
    nnls_solve_wave(M, p, ldm, K, r, r, w.RA, w.C + (int64_t)i * r, tol, lds, i, H + (int64_t)i * ldh,
                    resid2 != nullptr ? resid2 + i : nullptr, info != nullptr ? info + i : nullptr);
}

// Rank sweep: workgroup (i, r - 1) solves column i on the prefix K[0..r) with
// R_A and C of the rmax-column QR in prefix mode (their leading r x r block and
// first r rows are exactly the factors of that prefix) and the tolerance from
// the prefix's ||A||_1; e2[(r - 1) n + i] gets the squared residual of the
// column (NaN past the valid prefix), H the fit at rmax.
__global__ void __launch_bounds__(64) sweep_solve_kernel(const double* __restrict__ M, int p, int n, int ldm,
                                                         const int* __restrict__ K, int rmax, NnlsWork w, double* H,
                                                         int ldh, double* e2) {
    extern __shared__ double lds[];
    const int i = blockIdx.x;
    const int r = (int)blockIdx.y + 1;
    const int L = (int)threadIdx.x;
    double* out = e2 + (int64_t)(r - 1) * n + i;
    if (r > (int)w.anorm1[2]) {                // past SPA's picks
        if (L == 0) *out = __builtin_nan("");
        if (r == rmax && L < rmax) H[(int64_t)i * ldh + L] = __builtin_nan("");
        return;
    }
    const double* cn1 = w.anorm1 + 3;
    double a1 = 0.0;
    for (int c = 0; c < r; ++c) a1 = cn1[c] > a1 ? cn1[c] : a1;
    const double tol = 10.0 * DBL_EPSILON * a1 * (double)(p > r ? p : r);
    nnls_solve_wave(M, p, ldm, K, r, rmax, w.RA, w.C + (int64_t)i * rmax, tol, lds, i,
                    r == rmax ? H + (int64_t)i * ldh : nullptr, out, nullptr);
}

// resid[r - 1] = sum_i e2[(r - 1) n + i] / ||M||_F^2 (0 when M = 0; NaN past
// the valid prefix), the relative residual of Sec. 4 for every rank.
__global__ void __launch_bounds__(kThreads) sweep_finish_kernel(const double* __restrict__ M, int p, int n, int ldm,
                                                                int rmax, const double* __restrict__ e2,
                                                                double* resid) {
    __shared__ double sv[kThreads / 64];
    double m2 = 0.0;
    for (int el = threadIdx.x; el < p * n; el += kThreads) {
        const int j = el / p, i = el - j * p;
        const double mij = M[(int64_t)j * ldm + i];
        m2 += mij * mij;
    }
    const double T = block_sum(m2, sv);
    for (int r = threadIdx.x; r < rmax; r += kThreads) {
        double E = 0.0;
        for (int i = 0; i < n; ++i) E += e2[(int64_t)r * n + i];
        resid[r] = T > 0.0 ? E / T : (E == E ? 0.0 : E);
    }
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
    // one thread per entry (i, j), i fastest (p n <= 65536)
    double e2 = 0.0, m2 = 0.0;
    for (int el = threadIdx.x; el < p * n; el += kThreads) {
        const int j = el / p, i = el - j * p;
        const double mij = M[(int64_t)j * ldm + i];
        double e = mij;
        for (int q = 0; q < r; ++q) e -= M[(int64_t)K[q] * ldm + i] * H[(int64_t)j * ldh + q];
        e2 += e * e;
        m2 += mij * mij;
    }
    const double E = block_sum(e2, sv);
    const double T = block_sum(m2, sv);
    if (threadIdx.x == 0) *out = T > 0.0 ? E / T : 0.0;
}

// ---- greedy XRAY (Sec. 2.1) -------------------------------------------------------
// One pick: score_j = ||Res^T M(:, j)|| / ||M(:, j)|| over unpicked columns with
// ||M(:, j)|| > 0 (Res = M before the first pick), argmax, append to K.
// With XL, M (ld p | 1, odd: conflict-free column walks) and Res are read
// from LDS copies; with PAR as well, the n^2 dot products Res(:, c)^T M(:, j)
// are spread over the threads into an LDS table before thread j sums their
// squares.  Every sum keeps the order of the global version.
__host__ __device__ constexpr bool xray_in_lds(int p, int n) {
    return (size_t)((p | 1) + p) * n * sizeof(double) <= kLdsCap;
}
__host__ __device__ constexpr bool xray_pairs_in_lds(int p, int n) {
    return (size_t)((p | 1) + p + n) * n * sizeof(double) <= kLdsCap;
}
template <bool XL, bool PAR = false>
__global__ void __launch_bounds__(kThreads) xray_pick_kernel(const double* __restrict__ M, int p, int n, int ldm,
                                                             const double* __restrict__ Res, int t, int* K,
                                                             int* state) {
    extern __shared__ double xr_lds[];
    __shared__ double sv[kThreads / 64];
    __shared__ int si[kThreads / 64];
    if (state[0] != 0) return;                       // stopped earlier (uniform)
    const int lm = XL ? (p | 1) : ldm;
    const double* Mm = XL ? (const double*)xr_lds : M;
    const double* Rr = XL ? (const double*)(xr_lds + (size_t)lm * n) : Res;
    if constexpr (XL) {
        for (int e = threadIdx.x; e < p * n; e += kThreads) {
            const int c = e / p, i = e - c * p;
            xr_lds[c * lm + i] = M[(int64_t)c * ldm + i];
            xr_lds[(size_t)lm * n + e] = Res[e];
        }
        __syncthreads();
    }
    double* dt = xr_lds + (size_t)(lm + p) * n;       // PAR: d(c, j) at c n + j
    if constexpr (PAR) {
        for (int e = threadIdx.x; e < n * n; e += kThreads) {
            const int c = e / n, jj = e - c * n;
            const double* rc = Rr + (int64_t)c * p;
            const double* mj = Mm + (int64_t)jj * lm;
            double d = 0.0;
#pragma unroll 4
            for (int i = 0; i < p; ++i) d += rc[i] * mj[i];
            dt[e] = d;
        }
        __syncthreads();
    }
    const int j = threadIdx.x;
    double score = -DBL_MAX;
    if (j < n) {
        bool used = false;
        for (int q = 0; q < t; ++q) used = used || K[q] == j;
        const double* mj = Mm + (int64_t)j * lm;
        double mn = 0.0;
        for (int i = 0; i < p; ++i) mn += mj[i] * mj[i];
        if (!used && mn > 0.0) {
            double s2 = 0.0;
            for (int c = 0; c < n; ++c) {
                double d;
                if constexpr (PAR) {
                    d = dt[c * n + j];
                } else {
                    const double* rc = Rr + (int64_t)c * p;
                    d = 0.0;
#pragma unroll 4
                    for (int i = 0; i < p; ++i) d += rc[i] * mj[i];
                }
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
    return ((size_t)p * (r + n) + (size_t)r * r + (size_t)r * n + 3 + r) * 8 + 1024;
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
    return w;
}

int nnls_qr_launch(const double* M, int p, int n, int ldm, const int* K, int r, const NnlsWork& w,
                   hipStream_t stream) {
    // one wave when it has few columns per lane (its steps then need no
    // cross-wave sums or barriers), else kThreads
    if (nnls_aug_in_lds(p, n, r)) {
        const size_t lds = (size_t)nnls_qr_ld(p, true) * (r + n) * sizeof(double);
        if (r + n <= 128) {
            if (lds > 65536)
                TSNMF_HIP(hipFuncSetAttribute((const void*)nnls_qr_kernel<true, 64>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL((nnls_qr_kernel<true, 64>), dim3(1), dim3(64), lds, stream, M, p, n, ldm, K, r, w);
        } else {
            if (lds > 65536)
                TSNMF_HIP(hipFuncSetAttribute((const void*)nnls_qr_kernel<true, kThreads>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL((nnls_qr_kernel<true, kThreads>), dim3(1), dim3(kThreads), lds, stream, M, p, n, ldm,
                               K, r, w);
        }
    } else {
        hipLaunchKernelGGL((nnls_qr_kernel<false, kThreads>), dim3(1), dim3(kThreads), 0, stream, M, p, n, ldm, K, r,
                           w);
    }
    TSNMF_LAUNCH_CHECK();
    return TSNMF_OK;
}

int nnls_launch(const double* M, int p, int n, int ldm, const int* K, int r, double* H, int ldh, double* resid2,
                int* info, void* ws, hipStream_t stream, const int* skip = nullptr) {
    NnlsWork w = nnls_layout(ws, p, n, r);
    w.skip = skip;
    if (int st = nnls_qr_launch(M, p, n, ldm, K, r, w, stream)) return st;
    const size_t lds = nnls_solve_lds(r);
    if (lds > 65536)
        TSNMF_HIP(hipFuncSetAttribute((const void*)nnls_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds));
    hipLaunchKernelGGL(nnls_solve_kernel, dim3(n), dim3(64), lds, stream, M, p, n, ldm, K, r, w, H, ldh, resid2,
                       info);
    TSNMF_LAUNCH_CHECK();
    return TSNMF_OK;
}

}  // namespace

int select_spa_impl(const double* M, int p, int n, int ldm, const double* colscale, int r, int* K, double* score,
                    int* info, hipStream_t stream) {
    void* ws = nullptr;
    if (int st = workspace_get(kTicketBytes + (spa_z_in_lds(p, n) ? 0 : (size_t)p * n * 8), stream, &ws)) return st;
    double* Zg = (double*)((char*)ws + kTicketBytes);
    if (spa_z_in_lds(p, n)) {
        const size_t lds = (size_t)p * (n + 1) * sizeof(double);
        if (lds > 65536)
            TSNMF_HIP(hipFuncSetAttribute((const void*)spa_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lds));
        hipLaunchKernelGGL(spa_kernel<true>, dim3(1), dim3(kThreads), lds, stream, M, p, n, ldm, colscale, r, K,
                           score, info, Zg);
    } else {
        hipLaunchKernelGGL(spa_kernel<false>, dim3(1), dim3(kThreads), (size_t)p * sizeof(double), stream, M, p, n,
                           ldm, colscale, r, K, score, info, Zg);
    }
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

int rank_sweep_impl(const double* R, int p, int n, int ldr, const double* colscale, int rmax, int* K, double* H,
                    int ldh, double* resid, int* info, hipStream_t stream) {
    // SPA's picks for rmax are nested: the first r of them are SPA's picks
    // for r.  One QR of R(:, K) in prefix mode gives the factors of every
    // prefix; every (column, rank) pair is then solved in one launch and the
    // curve summed from the squared column residuals.  If SPA stops early, K
    // holds -1 past its picks and the ranks past them report NaN.
    if (int st = select_spa_impl(R, p, n, ldr, colscale, rmax, K, nullptr, info, stream)) return st;
    const size_t nb = nnls_bytes(p, n, rmax);
    void* ws = nullptr;
    if (int st = workspace_get(kTicketBytes + nb + (size_t)rmax * n * 8, stream, &ws)) return st;
    char* base = (char*)ws + kTicketBytes;
    NnlsWork w = nnls_layout(base, p, n, rmax);
    w.prefix = 1;
    double* e2 = (double*)(base + nb);
    if (int st = nnls_qr_launch(R, p, n, ldr, K, rmax, w, stream)) return st;
    const size_t lds = nnls_solve_lds(rmax);
    if (lds > 65536)
        TSNMF_HIP(hipFuncSetAttribute((const void*)sweep_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds));
    hipLaunchKernelGGL(sweep_solve_kernel, dim3(n, rmax), dim3(64), lds, stream, R, p, n, ldr, K, rmax, w, H, ldh,
                       e2);
    TSNMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(sweep_finish_kernel, dim3(1), dim3(kThreads), 0, stream, R, p, n, ldr, rmax, e2, resid);
    TSNMF_LAUNCH_CHECK();
    return TSNMF_OK;
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
    const bool xp = xray_pairs_in_lds(p, n);
    const bool xl = xray_in_lds(p, n);
    const size_t xl_lds = (size_t)((p | 1) + p + (xp ? n : 0)) * n * sizeof(double);
    if (xl && xl_lds > 65536)
        TSNMF_HIP(hipFuncSetAttribute(xp ? (const void*)xray_pick_kernel<true, true>
                                         : (const void*)xray_pick_kernel<true, false>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)xl_lds));
    hipLaunchKernelGGL(copy_matrix_kernel, dim3((unsigned)((pn + 255) / 256)), dim3(256), 0, stream, M, p, n, ldm,
                       Res);
    TSNMF_LAUNCH_CHECK();
    for (int t = 0; t < r && t < n; ++t) {
        if (xp)
            hipLaunchKernelGGL((xray_pick_kernel<true, true>), dim3(1), dim3(kThreads), xl_lds, stream, M, p, n, ldm,
                               Res, t, K, state);
        else if (xl)
            hipLaunchKernelGGL((xray_pick_kernel<true, false>), dim3(1), dim3(kThreads), xl_lds, stream, M, p, n, ldm,
                               Res, t, K, state);
        else
            hipLaunchKernelGGL(xray_pick_kernel<false>, dim3(1), dim3(kThreads), 0, stream, M, p, n, ldm, Res, t, K,
                               state);
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
