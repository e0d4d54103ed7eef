// HIP kernels for gfx950 (MI355X): the per-right-hand-side steps of the
// parallel sweep method.
//
// Mapping: one lane = one right-hand side (the series index n), one
// workgroup = one block j of rows x 256 consecutive right-hand sides.  With
// the RHS-interleaved layout F[i*N + n], every row access of a wavefront is
// one contiguous 256 B (FP32) or 512 B (FP64) span: loads and stores
// coalesce without any transposition.  The coefficients of the constant
// matrix are the same for every lane, so the sweep stages its block's rows
// of them in LDS and every lane reads them as broadcasts.
//
//   k_beta   eq. beta_symn: beta^R_j, beta^L_j of block j (FP64 accumulation).
//   k_iface  Theorem 2 (eq. theor_2): x at the interface rows by the two
//            first-order recurrences S^R_{k+1} = rho_k S^R_k + beta^R_k and
//            S^L_k = beta^L_k + lam_k S^L_{k+1}, x(s_k) = S^R_k + S^L_k.
//   k_sweep  Lemma 1 / Algorithm 1 step 3: the sweep inside each block with
//            both boundary values known.
#include "tdsolve.h"
#include "tds_internal.h"

namespace tds {

enum SweepKind { kSweep64 = 0, kSweepRefined = 1, kSweep32 = 2 };

// --------------------------------------------------------------------------
// beta weights (eq. beta_symn).  The weight arrays are read with
// wave-uniform addresses, which the compiler turns into scalar loads.
template <typename Fin>
__global__ __launch_bounds__(kWG) void k_beta(const Fin* __restrict__ F, int64_t N, int32_t P,
                                              const int64_t* __restrict__ starts,
                                              const double* __restrict__ wR,
                                              const double* __restrict__ wL,
                                              double* __restrict__ betaR,
                                              double* __restrict__ betaL) {
    const int32_t j = blockIdx.y;
    const int64_t lo = starts[j];
    const int t = (int)(starts[j + 1] - lo);
    const int64_t n = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (n >= N) return;
    const Fin* f = F + lo * N + n;
    double bR = 0.0, bL = 0.0;
    int r = 0;
    for (; r + 8 <= t; r += 8) {
        Fin v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = f[(int64_t)(r + u) * N];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double x = (double)v[u];
            bR = fma(wR[lo + r + u], x, bR);
            bL = fma(wL[lo + r + u], x, bL);
        }
    }
    for (; r < t; ++r) {
        const double x = (double)f[(int64_t)r * N];
        bR = fma(wR[lo + r], x, bR);
        bL = fma(wL[lo + r], x, bL);
    }
    if (j < P - 1) betaR[(int64_t)j * N + n] = bR;
    if (j > 0) betaL[(int64_t)j * N + n] = bL;
}

// --------------------------------------------------------------------------
// interface rows (Theorem 2).  xsep row k-1 holds x(s_k), k = 1..P-1.
__global__ __launch_bounds__(kWG) void k_iface(int64_t N, int32_t P,
                                               const double* __restrict__ rho,
                                               const double* __restrict__ lam,
                                               const double* __restrict__ betaR,
                                               const double* __restrict__ betaL,
                                               double* __restrict__ xsep) {
    const int64_t n = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (n >= N) return;
    double SR = betaR[n];                     // S^R_1 = beta^R_0
    xsep[n] = SR;
    for (int32_t k = 1; k <= P - 2; ++k) {    // S^R_{k+1}
        SR = fma(rho[k], SR, betaR[(int64_t)k * N + n]);
        xsep[(int64_t)k * N + n] = SR;
    }
    double SL = betaL[(int64_t)(P - 1) * N + n];   // S^L_{P-1} = beta^L_{P-1}
    xsep[(int64_t)(P - 2) * N + n] += SL;
    for (int32_t k = P - 2; k >= 1; --k) {    // S^L_k
        SL = fma(lam[k], SL, betaL[(int64_t)k * N + n]);
        xsep[(int64_t)(k - 1) * N + n] += SL;
    }
}

// --------------------------------------------------------------------------
// Block sweep, register-resident.  Block j's interior rows i0..i1 (block 0
// starts at row 0; the others at the row after their left interface row)
// are solved with x at the interface rows s_j (left) and s_{j+1} (right)
// known.  Each lane keeps its whole column of the block in VGPRs: F is read
// once and X written once.
template <int TMAX>
struct SweepLDS {
    double sub[TMAX], diag[TMAX], sup[TMAX], cp[TMAX], rd[TMAX];
    float sub32[TMAX], cp32[TMAX], rd32[TMAX];
};

// The row count CNT is a template constant for the common block sizes, so
// the unrolled row loops carry no per-row conditions; CNT == 0 takes the
// count at run time (rows past it are skipped by uniform branches).
template <int TMAX, int CNT, typename Fin, typename Xout, int KIND>
__device__ __forceinline__ void sweep_body(const Fin* __restrict__ fp, Xout* __restrict__ xp,
                                           int64_t N, int cnt_rt, double cl, double xl,
                                           double cr, double xr, const SweepLDS<TMAX>& L,
                                           float* __restrict__ my_f, int passes) {
    const int cnt = (CNT == 0) ? cnt_rt : CNT;
#define TDS_ACTIVE(r) ((CNT == 0) ? ((r) < cnt) : ((r) < CNT))
    Fin f[TMAX];
    {
        const Fin* q = fp;
#pragma unroll
        for (int r = 0; r < TMAX; ++r) {
            if (TDS_ACTIVE(r)) f[r] = *q;
            q += N;
        }
    }
    if constexpr (KIND == kSweepRefined) {
#pragma unroll
        for (int r = 0; r < TMAX; ++r)
            if (TDS_ACTIVE(r)) my_f[r * kWG] = (float)f[r];
    }

    // right-hand side of block row r with the known boundary values moved over
    auto g = [&](int r) -> double {
        double v = (KIND == kSweepRefined) ? (double)my_f[r * kWG] : (double)f[r];
        if (r == 0) v -= cl * xl;
        if (r == cnt - 1) v -= cr * xr;
        return v;
    };

    if constexpr (KIND == kSweep64) {
        double d[TMAX];
#pragma unroll
        for (int r = 0; r < TMAX; ++r) {
            if (TDS_ACTIVE(r)) {
                const double prev = (r > 0) ? d[r - 1] : 0.0;
                d[r] = (g(r) - L.sub[r] * prev) * L.rd[r];
            }
        }
        double x = 0.0;
        Xout* q = xp + (int64_t)(TMAX - 1) * N;
#pragma unroll
        for (int r = TMAX - 1; r >= 0; --r) {
            if (TDS_ACTIVE(r)) {
                x = d[r] - L.cp[r] * x;
                *q = (Xout)x;
            }
            q -= N;
        }
    } else if constexpr (KIND == kSweep32) {
        float w[TMAX];
#pragma unroll
        for (int r = 0; r < TMAX; ++r) {
            if (TDS_ACTIVE(r)) {
                const float prev = (r > 0) ? w[r - 1] : 0.0f;
                w[r] = ((float)g(r) - L.sub32[r] * prev) * L.rd32[r];
            }
        }
        float x = 0.0f;
        Xout* q = xp + (int64_t)(TMAX - 1) * N;
#pragma unroll
        for (int r = TMAX - 1; r >= 0; --r) {
            if (TDS_ACTIVE(r)) {
                x = w[r] - L.cp32[r] * x;
                *q = (Xout)x;
            }
            q -= N;
        }
    } else {
        // FP32 sweep, then `passes` times: FP64 residual of the block
        // system -> FP32 sweep of the residual -> FP64 update.
        double x[TMAX];
        float w[TMAX];
#pragma unroll
        for (int r = 0; r < TMAX; ++r) {
            if (TDS_ACTIVE(r)) {
                const float prev = (r > 0) ? w[r - 1] : 0.0f;
                w[r] = ((float)g(r) - L.sub32[r] * prev) * L.rd32[r];
            }
        }
        {
            float xs = 0.0f;
#pragma unroll
            for (int r = TMAX - 1; r >= 0; --r) {
                if (TDS_ACTIVE(r)) {
                    xs = w[r] - L.cp32[r] * xs;
                    x[r] = (double)xs;
                } else {
                    x[r] = 0.0;
                }
            }
        }
        for (int p = 0; p < passes; ++p) {
            // keep the LDS reads inside the pass: hoisting them out of the
            // loop would hold every row's coefficients in VGPRs
            asm volatile("" ::: "memory");
#pragma unroll
            for (int r = 0; r < TMAX; ++r) {
                if (TDS_ACTIVE(r)) {
                    double res = g(r) - L.diag[r] * x[r];
                    if (r > 0) res -= L.sub[r] * x[r - 1];
                    if (r + 1 < TMAX) res -= L.sup[r] * x[r + 1];
                    const float prev = (r > 0) ? w[r - 1] : 0.0f;
                    w[r] = ((float)res - L.sub32[r] * prev) * L.rd32[r];
                }
            }
            float dl = 0.0f;
#pragma unroll
            for (int r = TMAX - 1; r >= 0; --r) {
                if (TDS_ACTIVE(r)) {
                    dl = w[r] - L.cp32[r] * dl;
                    x[r] += (double)dl;
                }
            }
        }
        Xout* q = xp;
#pragma unroll
        for (int r = 0; r < TMAX; ++r) {
            if (TDS_ACTIVE(r)) *q = (Xout)x[r];
            q += N;
        }
    }
#undef TDS_ACTIVE
}

template <int TMAX, typename Fin, typename Xout, int KIND>
__global__ __launch_bounds__(kWG) void k_sweep_reg(
    const Fin* __restrict__ F, Xout* __restrict__ X, int64_t N, int32_t P,
    const int64_t* __restrict__ starts, const double* __restrict__ a64,
    const double* __restrict__ b64, const double* __restrict__ cp64,
    const double* __restrict__ rd64, const float* __restrict__ a32,
    const float* __restrict__ cp32, const float* __restrict__ rd32,
    const double* __restrict__ xsep, int passes) {
    __shared__ SweepLDS<TMAX> L;
    // the refined sweep keeps its FP32 input column in LDS (one row of 256
    // lanes per block row, conflict-free) so its VGPRs hold only x and the
    // FP32 elimination values
    __shared__ float s_f[KIND == kSweepRefined ? TMAX * kWG : 1];

    const int32_t j = blockIdx.y;
    const int64_t seg_lo = starts[j], seg_hi = starts[j + 1];
    const int64_t i0 = (j == 0) ? seg_lo : seg_lo + 1;
    const int cnt = (int)(seg_hi - i0);
    for (int r = threadIdx.x; r < cnt; r += kWG) {
        const int64_t i = i0 + r;
        L.sub[r] = (r > 0) ? a64[i - 1] : 0.0;
        L.sup[r] = (r < cnt - 1) ? a64[i] : 0.0;
        L.diag[r] = b64[i];
        L.cp[r] = cp64[i];
        L.rd[r] = rd64[i];
        L.sub32[r] = (r > 0) ? a32[i - 1] : 0.0f;
        L.cp32[r] = cp32[i];
        L.rd32[r] = rd32[i];
    }
    __syncthreads();

    const int64_t n = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (n >= N) return;
    const double xl = (j > 0) ? xsep[(int64_t)(j - 1) * N + n] : 0.0;
    const double xr = (j < P - 1) ? xsep[(int64_t)j * N + n] : 0.0;
    const double cl = (j > 0) ? a64[i0 - 1] : 0.0;        // A[i0][i0-1]
    const double cr = (j < P - 1) ? a64[seg_hi - 1] : 0.0; // A[i1][i1+1]
    if (j > 0) X[seg_lo * N + n] = (Xout)xl;

    const Fin* fp = F + i0 * N + n;
    Xout* xp = X + i0 * N + n;
    float* my_f = s_f + threadIdx.x;
    if (cnt == TMAX)
        sweep_body<TMAX, TMAX, Fin, Xout, KIND>(fp, xp, N, cnt, cl, xl, cr, xr, L, my_f, passes);
    else if (cnt == TMAX - 1)
        sweep_body<TMAX, TMAX - 1, Fin, Xout, KIND>(fp, xp, N, cnt, cl, xl, cr, xr, L, my_f,
                                                    passes);
    else
        sweep_body<TMAX, 0, Fin, Xout, KIND>(fp, xp, N, cnt, cl, xl, cr, xr, L, my_f, passes);
}

// --------------------------------------------------------------------------
// Block sweep for blocks longer than the register path holds: the forward
// elimination is kept in X itself and read back by the back substitution.
// FP64 arithmetic except for KIND == kSweep32.
template <typename Fin, typename Xout, int KIND>
__global__ __launch_bounds__(kWG) void k_sweep_stream(
    const Fin* __restrict__ F, Xout* __restrict__ X, int64_t N, int32_t P,
    const int64_t* __restrict__ starts, const double* __restrict__ a64,
    const double* __restrict__ cp64, const double* __restrict__ rd64,
    const double* __restrict__ xsep) {
    const int32_t j = blockIdx.y;
    const int64_t seg_lo = starts[j], seg_hi = starts[j + 1];
    const int64_t i0 = (j == 0) ? seg_lo : seg_lo + 1;
    const int64_t cnt = seg_hi - i0;
    const int64_t n = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (n >= N) return;
    const double xl = (j > 0) ? xsep[(int64_t)(j - 1) * N + n] : 0.0;
    const double xr = (j < P - 1) ? xsep[(int64_t)j * N + n] : 0.0;
    const double cl = (j > 0) ? a64[i0 - 1] : 0.0;
    const double cr = (j < P - 1) ? a64[seg_hi - 1] : 0.0;
    if (j > 0) X[seg_lo * N + n] = (Xout)xl;
    double prev = 0.0;
    for (int64_t r = 0; r < cnt; ++r) {
        const int64_t i = i0 + r;
        double v = (double)F[i * N + n];
        if (r == 0) v -= cl * xl;
        if (r == cnt - 1) v -= cr * xr;
        double d;
        if (KIND == kSweep32)
            d = (double)(((float)v - (float)(r > 0 ? a64[i - 1] : 0.0) * (float)prev) * (float)rd64[i]);
        else
            d = (v - (r > 0 ? a64[i - 1] : 0.0) * prev) * rd64[i];
        X[i * N + n] = (Xout)d;
        prev = d;
    }
    double x = 0.0;
    for (int64_t r = cnt - 1; r >= 0; --r) {
        const int64_t i = i0 + r;
        const double d = (double)X[i * N + n];
        if (KIND == kSweep32)
            x = (double)((float)d - (float)cp64[i] * (float)x);
        else
            x = d - cp64[i] * x;
        X[i * N + n] = (Xout)x;
    }
}

// --------------------------------------------------------------------------
// Residual metrics: per (row chunk, RHS) partials, then a per-RHS finish.
template <typename Fin, typename Xin>
__global__ __launch_bounds__(kWG) void k_resid_part(const Fin* __restrict__ F,
                                                    const Xin* __restrict__ X, int64_t N,
                                                    int64_t M, const double* __restrict__ a64,
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
        if (i > 0) r -= a64[i - 1] * (double)X[(i - 1) * N + n];
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
// Adjoint reductions over the series: one workgroup per row i, a fixed
// strided order per lane and a fixed LDS tree, so results are bitwise
// reproducible (no floating-point atomics).
template <typename Xin, typename Gin>
__global__ __launch_bounds__(kWG) void k_adjoint_reduce(const Xin* __restrict__ X,
                                                        const Gin* __restrict__ gF, int64_t N,
                                                        int64_t M, double* __restrict__ ga,
                                                        double* __restrict__ gb) {
    __shared__ double sa[kWG], sb[kWG];
    const int64_t i = blockIdx.x;
    double accb = 0.0, acca = 0.0;
    const bool has_next = (i + 1 < M);
    for (int64_t n = threadIdx.x; n < N; n += kWG) {
        const double x = (double)X[i * N + n];
        const double g = (double)gF[i * N + n];
        accb = fma(g, x, accb);
        if (has_next) {
            const double x1 = (double)X[(i + 1) * N + n];
            const double g1 = (double)gF[(i + 1) * N + n];
            acca = fma(g, x1, acca);
            acca = fma(g1, x, acca);
        }
    }
    sa[threadIdx.x] = acca;
    sb[threadIdx.x] = accb;
    __syncthreads();
    for (int w = kWG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sa[threadIdx.x] += sa[threadIdx.x + w];
            sb[threadIdx.x] += sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (gb) gb[i] = -sb[0];
        if (ga && has_next) ga[i] = -sa[0];
    }
}

// ==========================================================================
// launchers
static inline dim3 grid2(int64_t N, int64_t y) {
    return dim3((unsigned)((N + kWG - 1) / kWG), (unsigned)y, 1);
}

hipError_t launch_beta(const DevTables& t, const void* F, bool f32, int64_t N,
                       double* betaR, double* betaL, hipStream_t s) {
    if (t.P < 2 || N == 0) return hipSuccess;
    dim3 g = grid2(N, t.P);
    if (f32)
        hipLaunchKernelGGL(k_beta<float>, g, dim3(kWG), 0, s, (const float*)F, N, t.P,
                           t.starts, t.wR, t.wL, betaR, betaL);
    else
        hipLaunchKernelGGL(k_beta<double>, g, dim3(kWG), 0, s, (const double*)F, N, t.P,
                           t.starts, t.wR, t.wL, betaR, betaL);
    return hipGetLastError();
}

hipError_t launch_iface(const DevTables& t, const double* betaR, const double* betaL,
                        double* xsep, int64_t N, hipStream_t s) {
    if (t.P < 2 || N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iface, grid2(N, 1), dim3(kWG), 0, s, N, t.P, t.rho, t.lam, betaR,
                       betaL, xsep);
    return hipGetLastError();
}

template <int TMAX, typename Fin, typename Xout, int KIND>
static void go_reg(const DevTables& t, const void* F, void* X, int64_t N, int passes,
                   const double* xsep, hipStream_t s) {
    hipLaunchKernelGGL((k_sweep_reg<TMAX, Fin, Xout, KIND>), grid2(N, t.P), dim3(kWG), 0, s,
                       (const Fin*)F, (Xout*)X, N, t.P, t.starts, t.a64, t.b64, t.cp64, t.rd64,
                       t.a32, t.cp32, t.rd32, xsep, passes);
}

template <typename Fin, typename Xout, int KIND>
static void go_sized(const DevTables& t, const void* F, void* X, int64_t N, int passes,
                     const double* xsep, hipStream_t s) {
    const int m = t.max_rows;
    if (m <= 16)
        go_reg<16, Fin, Xout, KIND>(t, F, X, N, passes, xsep, s);
    else if (m <= 32)
        go_reg<32, Fin, Xout, KIND>(t, F, X, N, passes, xsep, s);
    else if (m <= 64)
        go_reg<64, Fin, Xout, KIND>(t, F, X, N, passes, xsep, s);
    else if (m <= kRegMaxRows && KIND != kSweepRefined)
        go_reg<128, Fin, Xout, KIND>(t, F, X, N, passes, xsep, s);
    else
        hipLaunchKernelGGL((k_sweep_stream<Fin, Xout, KIND == kSweep32 ? kSweep32 : kSweep64>),
                           grid2(N, t.P), dim3(kWG), 0, s, (const Fin*)F, (Xout*)X, N, t.P,
                           t.starts, t.a64, t.cp64, t.rd64, xsep);
}

hipError_t launch_sweep(const DevTables& t, const void* F, void* X, int64_t N, int mode,
                        int passes, const double* xsep, hipStream_t s) {
    if (N == 0) return hipSuccess;
    switch (mode) {
        case TDS_F64: go_sized<double, double, kSweep64>(t, F, X, N, passes, xsep, s); break;
        case TDS_F32_WIDE: go_sized<float, double, kSweep64>(t, F, X, N, passes, xsep, s); break;
        case TDS_F32: go_sized<float, float, kSweep32>(t, F, X, N, passes, xsep, s); break;
        case TDS_F32_REFINED:
            go_sized<float, double, kSweepRefined>(t, F, X, N, passes, xsep, s);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_residual(const DevTables& t, const void* F, const void* X, int64_t N,
                           int mode, double normA, double* part, double* out, hipStream_t s) {
    if (N == 0) return hipSuccess;
    const int64_t chunks = (t.M + kReduceRowChunk - 1) / kReduceRowChunk;
    dim3 g = grid2(N, chunks);
    switch (mode) {
        case TDS_F64:
            hipLaunchKernelGGL((k_resid_part<double, double>), g, dim3(kWG), 0, s,
                               (const double*)F, (const double*)X, N, t.M, t.a64, t.b64, part);
            break;
        case TDS_F32:
            hipLaunchKernelGGL((k_resid_part<float, float>), g, dim3(kWG), 0, s,
                               (const float*)F, (const float*)X, N, t.M, t.a64, t.b64, part);
            break;
        default:
            hipLaunchKernelGGL((k_resid_part<float, double>), g, dim3(kWG), 0, s,
                               (const float*)F, (const double*)X, N, t.M, t.a64, t.b64, part);
            break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_resid_finish, grid2(N, 1), dim3(kWG), 0, s, part, N, chunks, normA,
                       out);
    return hipGetLastError();
}

hipError_t launch_adjoint_reduce(const DevTables& t, const void* X, const void* gF, bool f32x,
                                 bool f32g, int64_t N, double* /*part*/, double* ga,
                                 double* gb, hipStream_t s) {
    if (N == 0 || (!ga && !gb)) return hipSuccess;
    dim3 g((unsigned)t.M, 1, 1);
    if (!f32x && !f32g)
        hipLaunchKernelGGL((k_adjoint_reduce<double, double>), g, dim3(kWG), 0, s,
                           (const double*)X, (const double*)gF, N, t.M, ga, gb);
    else if (!f32x && f32g)
        hipLaunchKernelGGL((k_adjoint_reduce<double, float>), g, dim3(kWG), 0, s,
                           (const double*)X, (const float*)gF, N, t.M, ga, gb);
    else if (f32x && f32g)
        hipLaunchKernelGGL((k_adjoint_reduce<float, float>), g, dim3(kWG), 0, s,
                           (const float*)X, (const float*)gF, N, t.M, ga, gb);
    else
        hipLaunchKernelGGL((k_adjoint_reduce<float, double>), g, dim3(kWG), 0, s,
                           (const float*)X, (const double*)gF, N, t.M, ga, gb);
    return hipGetLastError();
}

}  // namespace tds
