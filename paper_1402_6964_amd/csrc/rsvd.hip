// SVD of the n x n factor R (Sec. 3.1, "TSQR and R-SVD": with X = QR and
// R = U S V^T, X = (QU) S V^T, so the singular values and right singular
// vectors of X come from R) and the rank sweep of residuals in the reduced
// space (Sec. 2.2 and Sec. 2.4: selection, NNLS and residual all work on R,
// so the residual of many candidate ranks costs n x n work).
//
// The SVD is one-sided Jacobi (Hestenes) in FP64 on one workgroup: the
// columns of A = R are orthogonalised by plane rotations of column pairs,
// the same rotations accumulated in V, until every pair is orthogonal to
// working accuracy; then s_i = ||a_i||, u_i = a_i / s_i.  A sweep visits all
// pairs in n - 1 rounds of n / 2 disjoint pairs (round-robin order), one
// wave per pair at a time.  One-sided Jacobi determines small singular
// values to high relative accuracy.
#include <float.h>

#include "common.hpp"
#include "wave.hpp"

namespace tsnmf {

namespace {

constexpr int kSvdWaves = 8;
constexpr int kSvdMaxSweeps = 40;

// Pair k of round `rd` of the round-robin tournament on `np` (even) players:
// player 0 stays, the others rotate.
__device__ __forceinline__ void rr_pair(int np, int rd, int k, int* i, int* j) {
    auto pos = [&](int q) { return q == 0 ? 0 : 1 + (q - 1 + rd) % (np - 1); };
    *i = pos(k);
    *j = pos(np - 1 - k);
}

__global__ void __launch_bounds__(kSvdWaves * 64) rsvd_kernel(const double* __restrict__ R, int n, int ldr,
                                                             double* A, double* V, double* S, double* U, int ldu,
                                                             double* Vout, int ldv, int* info) {
    __shared__ double soff[kSvdWaves];
    __shared__ int sdone;
    __shared__ int sorder[256];
    const int tid = (int)threadIdx.x;
    const int wv = tid >> 6, L = tid & 63;
    for (int e = tid; e < n * n; e += kSvdWaves * 64) {
        const int r = e % n, c = e / n;
        A[(int64_t)c * n + r] = R[(int64_t)c * ldr + r];
        V[(int64_t)c * n + r] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    const int np = n + (n & 1);
    const double tol = (double)n * DBL_EPSILON;
    int sweeps = 0;
    for (; sweeps < kSvdMaxSweeps; ++sweeps) {
        double off = 0.0;
        for (int rd = 0; rd < np - 1; ++rd) {
            for (int k = wv; k < np / 2; k += kSvdWaves) {
                int i, j;
                rr_pair(np, rd, k, &i, &j);
                if (i >= n || j >= n) continue;
                if (i > j) { const int t = i; i = j; j = t; }
                double* ai = A + (int64_t)i * n;
                double* aj = A + (int64_t)j * n;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int r = L; r < n; r += 64) {
                    const double x = ai[r], y = aj[r];
                    al = __builtin_fma(x, x, al);
                    be = __builtin_fma(y, y, be);
                    ga = __builtin_fma(x, y, ga);
                }
                al = wave_sum(al);
                be = wave_sum(be);
                ga = wave_sum(ga);
                const double nrm = __builtin_sqrt(al * be);
                if (ga == 0.0 || !(__builtin_fabs(ga) > tol * nrm)) continue;
                off = fmax(off, __builtin_fabs(ga) / nrm);
                // rotation making columns i and j orthogonal: t = tan(theta),
                // the root of t^2 + 2 zeta t - 1 = 0 of smaller magnitude
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (__builtin_fabs(zeta) + __builtin_sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / __builtin_sqrt(1.0 + t * t);
                const double s = c * t;
                double* vi = V + (int64_t)i * n;
                double* vj = V + (int64_t)j * n;
                for (int r = L; r < n; r += 64) {
                    const double x = ai[r], y = aj[r];
                    ai[r] = c * x - s * y;
                    aj[r] = s * x + c * y;
                    const double p = vi[r], q = vj[r];
                    vi[r] = c * p - s * q;
                    vj[r] = s * p + c * q;
                }
            }
            __syncthreads();                       // pairs of the next round touch other columns
        }
        if (L == 0) soff[wv] = off;
        __syncthreads();
        if (tid == 0) {
            double m = 0.0;
            for (int q = 0; q < kSvdWaves; ++q) m = fmax(m, soff[q]);
            sdone = m <= tol;
        }
        __syncthreads();
        if (sdone) break;
    }
    // singular values, sorted descending (ties by index)
    double* norms = S;                              // reuse the output as scratch
    for (int c = wv; c < n; c += kSvdWaves) {
        double s2 = 0.0;
        for (int r = L; r < n; r += 64) s2 = __builtin_fma(A[(int64_t)c * n + r], A[(int64_t)c * n + r], s2);
        s2 = wave_sum(s2);
        if (L == 0) norms[c] = __builtin_sqrt(s2);
    }
    __syncthreads();
    for (int c = tid; c < n; c += kSvdWaves * 64) {
        const double sc = norms[c];
        int rank = 0;
        for (int q = 0; q < n; ++q) rank += norms[q] > sc || (norms[q] == sc && q < c);
        sorder[rank] = c;
    }
    __syncthreads();
    // n <= 256 < the workgroup's 512 threads: one value per thread
    const double mine = tid < n ? norms[sorder[tid]] : 0.0;
    __syncthreads();
    if (tid < n) S[tid] = mine;
    __syncthreads();
    // V and U columns in that order, each pair signed so that the
    // largest-magnitude entry of v is positive (first such entry on ties)
    for (int c = wv; c < n; c += kSvdWaves) {
        const int src = sorder[c];
        const double* vs = V + (int64_t)src * n;
        double best = -1.0;
        int bi = 0;
        for (int r = L; r < n; r += 64) {
            const double a = __builtin_fabs(vs[r]);
            if (a > best) { best = a; bi = r; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off);
            const int oi = __shfl_xor(bi, off);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        const double sg = vs[bi] < 0.0 ? -1.0 : 1.0;
        const double sc = S[c];
        for (int r = L; r < n; r += 64) {
            Vout[(int64_t)c * ldv + r] = sg * vs[r];
            if (U != nullptr) U[(int64_t)c * ldu + r] = sc > 0.0 ? sg * A[(int64_t)src * n + r] / sc : 0.0;
        }
    }
    if (tid == 0 && info != nullptr) *info = sweeps < kSvdMaxSweeps ? sweeps + 1 : -1;
}

}  // namespace

int rsvd_impl(const double* R, int n, int ldr, double* S, double* V, int ldv, double* U, int ldu, int* info,
              hipStream_t stream) {
    void* ws = nullptr;
    if (int st = workspace_get(kTicketBytes + 2 * (size_t)n * n * 8, stream, &ws)) return st;
    double* A = (double*)((char*)ws + kTicketBytes);
    double* Vw = A + (size_t)n * n;
    hipLaunchKernelGGL(rsvd_kernel, dim3(1), dim3(kSvdWaves * 64), 0, stream, R, n, ldr, A, Vw, S, U, ldu, V, ldv,
                       info);
    TSNMF_LAUNCH_CHECK();
    return TSNMF_OK;
}

}  // namespace tsnmf
