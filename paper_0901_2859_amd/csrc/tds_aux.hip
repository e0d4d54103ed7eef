// HIP kernels for gfx950 (MI355X) outside the solve itself: residual
// metrics of a computed solution and the reductions of the adjoint
// (gradients with respect to the matrix coefficients).
#include "tdsolve.h"
#include <algorithm>

#include "tds_internal.h"

namespace tds {

static inline dim3 grid2(int64_t N, int64_t y) {
    return dim3((unsigned)((N + kWG - 1) / kWG), (unsigned)y, 1);
}

// --------------------------------------------------------------------------
// Residual metrics: per (row chunk, RHS) partials, then a per-RHS finish.
template <typename Fin, typename Xin>
__global__ __launch_bounds__(kWG) void k_resid_part(const Fin* __restrict__ F,
                                                    const Xin* __restrict__ X, int64_t N,
                                                    int64_t M, const double* __restrict__ a64,
                                                    const double* __restrict__ l64,
                                                    const double* __restrict__ b64,
                                                    double* __restrict__ part) {
    const int64_t n = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (n >= N) return;
    const int64_t lo = c * kReduceRowChunk;
    const int64_t hi = (lo + kReduceRowChunk < M) ? lo + kReduceRowChunk : M;
    double rmx = 0.0, r2 = 0.0, xmx = 0.0, fmx = 0.0, f2 = 0.0;
    for (int64_t i = lo; i < hi; ++i) {
        const double x = (double)X[i * N + n];
        double r = (double)F[i * N + n] - b64[i] * x;
        if (i > 0) r -= l64[i - 1] * (double)X[(i - 1) * N + n];
        if (i + 1 < M) r -= a64[i] * (double)X[(i + 1) * N + n];
        const double f = (double)F[i * N + n];
        rmx = fmax(rmx, fabs(r));
        r2 += r * r;
        xmx = fmax(xmx, fabs(x));
        fmx = fmax(fmx, fabs(f));
        f2 += f * f;
    }
    double* p = part + (c * 5) * N + n;
    p[0] = rmx;
    p[N] = r2;
    p[2 * N] = xmx;
    p[3 * N] = fmx;
    p[4 * N] = f2;
}

__global__ __launch_bounds__(kWG) void k_resid_finish(const double* __restrict__ part, int64_t N,
                                                      int64_t chunks, double normA,
                                                      double* __restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (n >= N) return;
    double rmx = 0.0, r2 = 0.0, xmx = 0.0, fmx = 0.0, f2 = 0.0;
    for (int64_t c = 0; c < chunks; ++c) {
        const double* p = part + (c * 5) * N + n;
        rmx = fmax(rmx, p[0]);
        r2 += p[N];
        xmx = fmax(xmx, p[2 * N]);
        fmx = fmax(fmx, p[3 * N]);
        f2 += p[4 * N];
    }
    const double den = normA * xmx + fmx;
    out[n] = den > 0.0 ? rmx / den : 0.0;
    out[N + n] = f2 > 0.0 ? sqrt(r2) / sqrt(f2) : sqrt(r2);
}

// --------------------------------------------------------------------------
// Adjoint reductions over the series: one workgroup per kAdjRows rows
// i0 .. i0 + kAdjRows - 1, which reads rows i0 .. i0 + kAdjRows of X and gF
// once each (row i + 1 serves both ga_i and gb_{i+1}), so the kernel moves
// (1 + 1 / kAdjRows) times the bytes of X and gF.  Every lane sums its
// right-hand sides n = lane, lane + 256, ... in that order, then a fixed LDS
// tree adds the lanes: results are bitwise reproducible (no floating-point
// atomics).  g32 (may be null) receives rows of gF rounded to FP32 on the
// way.
constexpr int kAdjRows = 4;

template <typename Xin, typename Gin>
__global__ __launch_bounds__(kWG) void k_adjoint_reduce(const Xin* __restrict__ X,
                                                        const Gin* __restrict__ gF, int64_t N,
                                                        int64_t M, float* __restrict__ g32,
                                                        double* __restrict__ ga,
                                                        double* __restrict__ gb) {
    __shared__ double sa[kAdjRows][kWG], sb[kAdjRows][kWG];
    const int64_t i0 = (int64_t)blockIdx.x * kAdjRows;
    const int rows = (int)min<int64_t>(kAdjRows, M - i0);       // rows reduced here
    double acca[kAdjRows], accb[kAdjRows];
#pragma unroll
    for (int r = 0; r < kAdjRows; ++r) acca[r] = accb[r] = 0.0;
    for (int64_t n = threadIdx.x; n < N; n += kWG) {
        double x[kAdjRows + 1], g[kAdjRows + 1];
#pragma unroll
        for (int r = 0; r <= kAdjRows; ++r) {
            // rows past the matrix (and row i0 + kAdjRows past M) are zero
            const bool in = r < rows || (r == rows && i0 + r < M);
            x[r] = in ? (double)X[(i0 + r) * N + n] : 0.0;
            g[r] = in ? (double)gF[(i0 + r) * N + n] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < kAdjRows; ++r) {
            if (r < rows) {
                if (g32) g32[(i0 + r) * N + n] = (float)g[r];
                accb[r] = fma(g[r], x[r], accb[r]);
                acca[r] = fma(g[r], x[r + 1], acca[r]);
                acca[r] = fma(g[r + 1], x[r], acca[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kAdjRows; ++r) {
        sa[r][threadIdx.x] = acca[r];
        sb[r][threadIdx.x] = accb[r];
    }
    __syncthreads();
    for (int w = kWG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int r = 0; r < kAdjRows; ++r) {
                sa[r][threadIdx.x] += sa[r][threadIdx.x + w];
                sb[r][threadIdx.x] += sb[r][threadIdx.x + w];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < rows) {
        const int64_t i = i0 + threadIdx.x;
        if (gb) gb[i] = -sb[threadIdx.x][0];
        if (ga && i + 1 < M) ga[i] = -sa[threadIdx.x][0];
    }
}

// --------------------------------------------------------------------------
// Scaled strided copy of an S x M x L array through 64 x 64 LDS tiles of
// (s, l) per i: the reads walk l fastest, the writes walk s fastest, so a
// layout change between (s, i, l) and (l, i, s) moves whole rows on both
// sides.  Grid: (tiles of l x tiles of s, M).
constexpr int kCopyTile = 64;

template <typename T>
__global__ __launch_bounds__(kWG) void k_strided_copy(const T* __restrict__ src, T* __restrict__ dst,
                                                      int64_t S, int64_t L, int64_t ss0,
                                                      int64_t ss1, int64_t ss2, int64_t ds0,
                                                      int64_t ds1, int64_t ds2, T alpha) {
    __shared__ T tile[kCopyTile][kCopyTile + 1];
    const int64_t tl = (L + kCopyTile - 1) / kCopyTile;
    const int64_t l0 = (int64_t)(blockIdx.x % tl) * kCopyTile;
    const int64_t s0 = (int64_t)(blockIdx.x / tl) * kCopyTile;
    const int64_t i = blockIdx.y;
    const int c = threadIdx.x % kCopyTile, r0 = threadIdx.x / kCopyTile;   // 4 rows per pass
    constexpr int kRows = kWG / kCopyTile;
#pragma unroll 4
    for (int r = r0; r < kCopyTile; r += kRows) {
        const int64_t s = s0 + r, l = l0 + c;
        if (s < S && l < L) tile[r][c] = src[s * ss0 + i * ss1 + l * ss2];
    }
    __syncthreads();
#pragma unroll 4
    for (int r = r0; r < kCopyTile; r += kRows) {
        const int64_t l = l0 + r, s = s0 + c;
        if (s < S && l < L) dst[s * ds0 + i * ds1 + l * ds2] = alpha * tile[c][r];
    }
}

// ==========================================================================
// launchers
hipError_t launch_residual(const DevTables& t, const void* F, const void* X, int64_t N,
                           int mode, double normA, double* part, double* out, hipStream_t s) {
    if (N == 0) return hipSuccess;
    const int64_t chunks = (t.M + kReduceRowChunk - 1) / kReduceRowChunk;
    dim3 g = grid2(N, chunks);
    switch (mode) {
        case TDS_F64:
            hipLaunchKernelGGL((k_resid_part<double, double>), g, dim3(kWG), 0, s,
                               (const double*)F, (const double*)X, N, t.M, t.a64, t.l64, t.b64, part);
            break;
        case TDS_F32:
            hipLaunchKernelGGL((k_resid_part<float, float>), g, dim3(kWG), 0, s,
                               (const float*)F, (const float*)X, N, t.M, t.a64, t.l64, t.b64, part);
            break;
        default:
            hipLaunchKernelGGL((k_resid_part<float, double>), g, dim3(kWG), 0, s,
                               (const float*)F, (const double*)X, N, t.M, t.a64, t.l64, t.b64, part);
            break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_resid_finish, grid2(N, 1), dim3(kWG), 0, s, part, N, chunks, normA,
                       out);
    return hipGetLastError();
}

hipError_t launch_adjoint_reduce(const DevTables& t, const void* X, const void* gF, bool f32x,
                                 bool f32g, int64_t N, float* g32, double* ga, double* gb,
                                 hipStream_t s) {
    if (N == 0 || (!ga && !gb && !g32)) return hipSuccess;
    dim3 g((unsigned)((t.M + kAdjRows - 1) / kAdjRows), 1, 1);
    if (!f32x && !f32g)
        hipLaunchKernelGGL((k_adjoint_reduce<double, double>), g, dim3(kWG), 0, s,
                           (const double*)X, (const double*)gF, N, t.M, g32, ga, gb);
    else if (!f32x && f32g)
        hipLaunchKernelGGL((k_adjoint_reduce<double, float>), g, dim3(kWG), 0, s,
                           (const double*)X, (const float*)gF, N, t.M, g32, ga, gb);
    else if (f32x && f32g)
        hipLaunchKernelGGL((k_adjoint_reduce<float, float>), g, dim3(kWG), 0, s,
                           (const float*)X, (const float*)gF, N, t.M, g32, ga, gb);
    else
        hipLaunchKernelGGL((k_adjoint_reduce<float, double>), g, dim3(kWG), 0, s,
                           (const float*)X, (const double*)gF, N, t.M, g32, ga, gb);
    return hipGetLastError();
}

// Counter-based uniform[-1, 1) fill (splitmix64 of the element index and a
// seed) for timing runs that need right-hand sides but no host data.
template <typename T>
__global__ void k_fill_uniform(T* __restrict__ p, int64_t n, uint64_t seed) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        p[i] = (T)((double)(z >> 11) * 0x1.0p-52 - 1.0);
    }
}

hipError_t launch_fill_uniform(void* p, int64_t n, bool f32, uint64_t seed, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + kWG - 1) / kWG, 8192);
    if (f32)
        hipLaunchKernelGGL(k_fill_uniform<float>, dim3(blocks), dim3(kWG), 0, s, (float*)p, n, seed);
    else
        hipLaunchKernelGGL(k_fill_uniform<double>, dim3(blocks), dim3(kWG), 0, s, (double*)p, n,
                           seed);
    return hipGetLastError();
}

hipError_t launch_strided_copy(const void* src, void* dst, bool f64, int64_t S, int64_t M,
                               int64_t L, const int64_t* ss, const int64_t* ds, double alpha,
                               hipStream_t s) {
    if (S == 0 || M == 0 || L == 0) return hipSuccess;
    const int64_t tiles = ((L + kCopyTile - 1) / kCopyTile) * ((S + kCopyTile - 1) / kCopyTile);
    if (tiles > 0x7fffffffLL || M > 65535) return hipErrorInvalidValue;
    const dim3 g((unsigned)tiles, (unsigned)M, 1);
    if (f64)
        hipLaunchKernelGGL(k_strided_copy<double>, g, dim3(kWG), 0, s, (const double*)src,
                           (double*)dst, S, L, ss[0], ss[1], ss[2], ds[0], ds[1], ds[2], alpha);
    else
        hipLaunchKernelGGL(k_strided_copy<float>, g, dim3(kWG), 0, s, (const float*)src,
                           (float*)dst, S, L, ss[0], ss[1], ss[2], ds[0], ds[1], ds[2],
                           (float)alpha);
    return hipGetLastError();
}

}  // namespace tds
