// HIP kernels for gfx950 (MI355X): the per-right-hand-side steps of the
// parallel sweep method.
//
// Mapping: one lane = one right-hand side (the series index n), one
// workgroup = one block j of rows x 256 consecutive right-hand sides.  With
// the RHS-interleaved layout F[i*N + n], every row access of a wavefront is
// one contiguous 256 B (FP32) or 512 B (FP64) span: loads and stores
// coalesce without any transposition.  The coefficients of the constant
// matrix are the same for every lane: the beta kernel stages its block's
// weights in LDS, the sweep reads its coefficients through scalar loads;
// either way every lane gets them as broadcasts.
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
// beta weights (eq. beta_symn).  Workgroup (tile, j): block j of rows x 256
// consecutive right-hand sides, one per lane.  All rows of the block are
// loaded before any arithmetic (one round trip to memory per workgroup);
// rows past the block re-read its last row and get weight zero.  The
// weights are wave-uniform and come in through scalar loads.
template <int TMAX, typename Fin>
__global__ __launch_bounds__(kWG) void k_beta(const Fin* __restrict__ F, int64_t N, int32_t P,
                                              const int64_t* __restrict__ starts,
                                              const double* __restrict__ wR,
                                              const double* __restrict__ wL,
                                              const double2* __restrict__ wpad,
                                              double* __restrict__ betaR,
                                              double* __restrict__ betaL) {
    const int32_t j = blockIdx.y;
    const int64_t lo = starts[j];
    const int t = (int)(starts[j + 1] - lo);
    const int64_t n = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (n >= N) return;
    const Fin* f = F + lo * N + n;
    double bR = 0.0, bL = 0.0;
    if constexpr (TMAX > 0) {
        // weights zero-padded per block: rows past the end add nothing
        const double2* __restrict__ w = wpad + (int64_t)j * TMAX;
        Fin v[TMAX];
#pragma unroll
        for (int r = 0; r < TMAX; ++r) v[r] = f[(int64_t)(r < t ? r : t - 1) * N];
#pragma unroll
        for (int r = 0; r < TMAX; ++r) {
            const double2 c = w[r];
            bR = fma(c.x, (double)v[r], bR);
            bL = fma(c.y, (double)v[r], bL);
        }
    } else {
        const double* __restrict__ gR = wR + lo;
        const double* __restrict__ gL = wL + lo;
        constexpr int U = 16;
        int r = 0;
        for (; r + U <= t; r += U) {
            Fin v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = f[(int64_t)(r + u) * N];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                bR = fma(gR[r + u], (double)v[u], bR);
                bL = fma(gL[r + u], (double)v[u], bL);
            }
        }
        for (; r < t; ++r) {
            const double v = (double)f[(int64_t)r * N];
            bR = fma(gR[r], v, bR);
            bL = fma(gL[r], v, bL);
        }
    }
    if (j < P - 1) betaR[(int64_t)j * N + n] = bR;
    if (j > 0) betaL[(int64_t)j * N + n] = bL;
}

// --------------------------------------------------------------------------
// Interface step (Theorem 2): the O(P) recurrences
//   forward   y_j = rho_j y_{j-1} + beta^R_j,  j = 0..P-2 (y_{-1} = 0),
//             so that S^R_{k} = y_{k-1};
//   backward  z_j = lam_j z_{j+1} + beta^L_j,  j = P-1..1 (z_P = 0),
//             so that S^L_k = z_k;
//   x(s_k) = S^R_k + S^L_k, k = 1..P-1  (xsep row k-1),
// evaluated as a two-level scan: workgroup = 64 right-hand sides x G groups
// of consecutive blocks; each thread scans its group with zero input, the
// group carries (product of the factors, partial value) are combined through
// LDS, then each thread redoes its group with the true input.
constexpr int kScanRhs = 64;
constexpr int kScanMaxGroups = 16;

__global__ __launch_bounds__(kScanRhs * kScanMaxGroups) void k_iface(
    int64_t N, int32_t P, int32_t per, const double* __restrict__ rho,
    const double* __restrict__ lam, const double* __restrict__ betaR,
    const double* __restrict__ betaL, double* __restrict__ xsep) {
    __shared__ double s_carry[2][kScanMaxGroups][kScanRhs];
    __shared__ double s_prod[2][kScanMaxGroups];
    const int lane = threadIdx.x % kScanRhs;
    const int g = threadIdx.x / kScanRhs;
    const int64_t n = (int64_t)blockIdx.x * kScanRhs + lane;
    const bool live = n < N;
    // forward groups over j = 0..P-2, backward groups over j = 1..P-1
    const int32_t f0 = g * per, f1 = min(f0 + per, P - 1);
    const int32_t b1 = P - 1 - g * per, b0 = max(b1 - per, 0);   // j in (b0, b1]

    double yl = 0.0, pr = 1.0;
#pragma unroll 4
    for (int32_t j = f0; j < f1; ++j) {
        const double r = (j > 0) ? rho[j] : 0.0;
        yl = fma(r, yl, live ? betaR[(int64_t)j * N + n] : 0.0);
        pr *= r;
    }
    double zl = 0.0, pl = 1.0;
#pragma unroll 4
    for (int32_t j = b1; j > b0; --j) {
        const double l = (j < P - 1) ? lam[j] : 0.0;
        zl = fma(l, zl, live ? betaL[(int64_t)j * N + n] : 0.0);
        pl *= l;
    }
    s_carry[0][g][lane] = yl;
    s_carry[1][g][lane] = zl;
    if (lane == 0) {
        s_prod[0][g] = (f0 < f1) ? pr : 1.0;
        s_prod[1][g] = (b0 < b1) ? pl : 1.0;
    }
    __syncthreads();
    double yin = 0.0, zin = 0.0;
    for (int q = 0; q < g; ++q) yin = fma(s_prod[0][q], yin, s_carry[0][q][lane]);
    for (int q = 0; q < g; ++q) zin = fma(s_prod[1][q], zin, s_carry[1][q][lane]);
    // redo the forward group with its true input: y_j = S^R_{j+1} into xsep
    if (live) {
        double y = yin;
#pragma unroll 4
        for (int32_t j = f0; j < f1; ++j) {
            const double r = (j > 0) ? rho[j] : 0.0;
            y = fma(r, y, betaR[(int64_t)j * N + n]);
            xsep[(int64_t)j * N + n] = y;
        }
    }
    __syncthreads();    // S^R of every group is in xsep (same workgroup)
    if (!live) return;
    double z = zin;
#pragma unroll 4
    for (int32_t j = b1; j > b0; --j) {
        const double l = (j < P - 1) ? lam[j] : 0.0;
        z = fma(l, z, betaL[(int64_t)j * N + n]);
        xsep[(int64_t)(j - 1) * N + n] += z;           // x(s_j) = S^R_j + S^L_j
    }
}

// --------------------------------------------------------------------------
// Block sweep, register-resident.  Block j's interior rows i0..i1 (block 0
// starts at row 0; the others at the row after their left interface row)
// are solved with x at the interface rows s_j (left, xl) and s_{j+1}
// (right, xr) known (Lemma 1).  Each lane keeps its whole column of the
// block in VGPRs: F is read once and X written once.
//
// The coefficients are the same for every lane; they are read through
// wave-uniform addresses, i.e. scalar loads into SGPRs through the scalar
// cache, which broadcast to the wavefront without occupying VGPRs.  The
// tables are separate arrays so that each sweep fetches only the bytes it
// uses (the scalar fetch volume per row shows directly in the run time).
//
// One kernel serves every block length cnt <= TMAX: rows cnt..TMAX-1 are
// "phantom" rows.  They re-read the block's last real row of F and the
// (padded, always in-bounds) table rows that follow, so their values stay
// finite, and they never feed back into real rows because the last real
// row's elimination factor and block-interior coupling are zero.  They are
// not stored.
struct BlockCoef {
    // tables offset to the block's first interior row i0; valid up to
    // i0 + TMAX (the device tables carry kRegMaxRows padding rows)
    const double* __restrict__ a64;
    const double* __restrict__ b64;
    const double* __restrict__ cp64;
    const double* __restrict__ rd64;
    const double* __restrict__ in64;
    const double* __restrict__ u;
    const double* __restrict__ v;
    const float* __restrict__ a32;
    const float* __restrict__ cp32;
    const float* __restrict__ rd32;
    const float* __restrict__ in32;
};

template <int TMAX, typename Fin, typename Xout, int KIND>
__device__ __forceinline__ void sweep_body(const Fin* __restrict__ fp, Xout* __restrict__ xp,
                                           int64_t N, int cnt, double cl, double xl, double cr,
                                           double xr, const BlockCoef& L,
                                           float* __restrict__ my_f, int passes) {
    Fin f[TMAX];
#pragma unroll
    for (int r = 0; r < TMAX; ++r) f[r] = fp[(int64_t)(r < cnt ? r : cnt - 1) * N];

    if constexpr (KIND == kSweep64 || KIND == kSweep32) {
        // one pass: the known boundary values are moved to the right-hand
        // side of the block's first and last interior rows
        const double clxl = cl * xl, crxr = cr * xr;
        auto g = [&](int r) -> double {
            double val = (double)f[r];
            if (r == 0) val -= clxl;
            if (r == cnt - 1) val -= crxr;
            return val;
        };
        if constexpr (KIND == kSweep64) {
            double d[TMAX];
#pragma unroll
            for (int r = 0; r < TMAX; ++r) {
                const double prev = (r > 0) ? d[r - 1] : 0.0;
                const double sub = (r > 0) ? L.a64[r - 1] : 0.0;
                d[r] = (g(r) - sub * prev) * L.rd64[r];
            }
            double x = 0.0;
            Xout* q = xp + (int64_t)(TMAX - 1) * N;
#pragma unroll
            for (int r = TMAX - 1; r >= 0; --r) {
                x = d[r] - L.cp64[r] * x;
                if (r < cnt) *q = (Xout)x;
                q -= N;
            }
        } else {
            float w[TMAX];
#pragma unroll
            for (int r = 0; r < TMAX; ++r) {
                const float prev = (r > 0) ? w[r - 1] : 0.0f;
                const float sub = (r > 0) ? L.a32[r - 1] : 0.0f;
                w[r] = ((float)g(r) - sub * prev) * L.rd32[r];
            }
            float x = 0.0f;
            Xout* q = xp + (int64_t)(TMAX - 1) * N;
#pragma unroll
            for (int r = TMAX - 1; r >= 0; --r) {
                x = w[r] - L.cp32[r] * x;
                if (r < cnt) *q = (Xout)x;
                q -= N;
            }
        }
    } else {
        // Refined: the block is solved with zero boundary values, x0 =
        // T^{-1} f, by an FP32 sweep and then `passes` times FP64 residual
        // -> FP32 sweep of the residual -> FP64 update; the interface values
        // enter at the end by superposition, x = x0 + xl u + xr v.  (With
        // the boundary terms inside the right-hand side every pass would
        // carry a row-dependent condition.)
#pragma unroll
        for (int r = 0; r < TMAX; ++r) my_f[r * kWG] = (float)f[r];
        double x[TMAX];
        float w[TMAX];
#pragma unroll
        for (int r = 0; r < TMAX; ++r) {
            if ((r & 3) == 0) __builtin_amdgcn_sched_barrier(0);
            const float prev = (r > 0) ? w[r - 1] : 0.0f;
            const float sub = (r > 0) ? L.in32[r - 1] : 0.0f;
            w[r] = (my_f[r * kWG] - sub * prev) * L.rd32[r];
        }
        {
            float xs = 0.0f;
#pragma unroll
            for (int r = TMAX - 1; r >= 0; --r) {
                if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                xs = w[r] - L.cp32[r] * xs;
                x[r] = (double)xs;
            }
        }
        for (int p = 0; p < passes; ++p) {
            // keep the LDS reads of F and the table loads inside the pass:
            // an offset the compiler cannot see through stops it from
            // hoisting every row's coefficients out of the loop
            asm volatile("" ::: "memory");
            int z;
            asm volatile("s_mov_b32 %0, 0" : "=s"(z));
            const double* __restrict__ in64 = L.in64 + z;
            const double* __restrict__ b64 = L.b64 + z;
            const float* __restrict__ in32 = L.in32 + z;
            const float* __restrict__ cp32 = L.cp32 + z;
            const float* __restrict__ rd32 = L.rd32 + z;
#pragma unroll
            for (int r = 0; r < TMAX; ++r) {
                // bound the scheduler's look-ahead: the residuals do not
                // depend on the elimination chain, and computing them all
                // ahead of it would hold 64 FP64 values in registers
                if ((r & 3) == 0) __builtin_amdgcn_sched_barrier(0);
                double res = (double)my_f[r * kWG] - b64[r] * x[r];
                if (r > 0) res -= in64[r - 1] * x[r - 1];
                if (r + 1 < TMAX) res -= in64[r] * x[r + 1];
                const float prev = (r > 0) ? w[r - 1] : 0.0f;
                const float sub = (r > 0) ? in32[r - 1] : 0.0f;
                w[r] = ((float)res - sub * prev) * rd32[r];
            }
            float dl = 0.0f;
#pragma unroll
            for (int r = TMAX - 1; r >= 0; --r) {
                if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                dl = w[r] - cp32[r] * dl;
                x[r] += (double)dl;
            }
        }
        Xout* q = xp;
#pragma unroll
        for (int r = 0; r < TMAX; ++r) {
            if (r < cnt) *q = (Xout)fma(xr, L.v[r], fma(xl, L.u[r], x[r]));
            q += N;
        }
    }
}

// Occupancy target (waves per SIMD) of the refined sweep, which holds about
// 3 registers per row (x in FP64, the FP32 elimination value; F sits in
// LDS); the other sweeps are left to the compiler.
template <int KIND, int TMAX>
constexpr int sweep_min_waves() {
    return TMAX > 64 ? 1 : KIND == kSweepRefined ? 2 : 1;
}

// (The tables come in as separate __restrict__ parameters, not as one
// struct: only then can the compiler prove them unaliased by the stores to X
// and fetch them with scalar loads.)
template <int TMAX, typename Fin, typename Xout, int KIND>
__global__ __launch_bounds__(kWG, (sweep_min_waves<KIND, TMAX>())) void k_sweep_reg(
    const Fin* __restrict__ F, Xout* __restrict__ X, int64_t N, int32_t P,
    const int64_t* __restrict__ starts, const double* __restrict__ a64,
    const double* __restrict__ b64, const double* __restrict__ cp64,
    const double* __restrict__ rd64, const double* __restrict__ in64,
    const double* __restrict__ u, const double* __restrict__ v,
    const float* __restrict__ a32, const float* __restrict__ cp32,
    const float* __restrict__ rd32, const float* __restrict__ in32,
    const double* __restrict__ xsep, int passes) {
    // the refined sweep keeps its FP32 input column in LDS (one row of 256
    // lanes per block row, conflict-free) so that its VGPRs hold only x and
    // the FP32 elimination values
    __shared__ float s_f[KIND == kSweepRefined ? TMAX * kWG : 1];

    const int32_t j = blockIdx.y;
    const int64_t seg_lo = starts[j], seg_hi = starts[j + 1];
    const int64_t i0 = (j == 0) ? seg_lo : seg_lo + 1;
    const int cnt = (int)(seg_hi - i0);
    const int64_t n = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (n >= N) return;
    const double xl = (j > 0) ? xsep[(int64_t)(j - 1) * N + n] : 0.0;
    const double xr = (j < P - 1) ? xsep[(int64_t)j * N + n] : 0.0;
    const double cl = (j > 0) ? a64[i0 - 1] : 0.0;         // A[i0][i0-1]
    const double cr = (j < P - 1) ? a64[seg_hi - 1] : 0.0; // A[i1][i1+1]
    if (j > 0) X[seg_lo * N + n] = (Xout)xl;

    const BlockCoef C{a64 + i0, b64 + i0, cp64 + i0, rd64 + i0, in64 + i0, u + i0,
                      v + i0, a32 + i0, cp32 + i0, rd32 + i0, in32 + i0};
    sweep_body<TMAX, Fin, Xout, KIND>(F + i0 * N + n, X + i0 * N + n, N, cnt, cl, xl, cr, xr, C,
                                      s_f + threadIdx.x, passes);
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

template <typename Fin>
static void go_beta(const DevTables& t, const void* F, int64_t N, double* betaR, double* betaL,
                    hipStream_t s) {
    const dim3 g = grid2(N, t.P);
    switch (t.wpad_rows) {
        case 32:
            hipLaunchKernelGGL((k_beta<32, Fin>), g, dim3(kWG), 0, s, (const Fin*)F, N, t.P,
                               t.starts, t.wR, t.wL, t.wpad, betaR, betaL);
            break;
        case 64:
            hipLaunchKernelGGL((k_beta<64, Fin>), g, dim3(kWG), 0, s, (const Fin*)F, N, t.P,
                               t.starts, t.wR, t.wL, t.wpad, betaR, betaL);
            break;
        case 128:
            hipLaunchKernelGGL((k_beta<128, Fin>), g, dim3(kWG), 0, s, (const Fin*)F, N, t.P,
                               t.starts, t.wR, t.wL, t.wpad, betaR, betaL);
            break;
        default:
            hipLaunchKernelGGL((k_beta<0, Fin>), g, dim3(kWG), 0, s, (const Fin*)F, N, t.P,
                               t.starts, t.wR, t.wL, t.wpad, betaR, betaL);
    }
}

hipError_t launch_beta(const DevTables& t, const void* F, bool f32, int64_t N, double* betaR,
                       double* betaL, hipStream_t s) {
    if (t.P < 2 || N == 0) return hipSuccess;
    if (f32)
        go_beta<float>(t, F, N, betaR, betaL, s);
    else
        go_beta<double>(t, F, N, betaR, betaL, s);
    return hipGetLastError();
}

hipError_t launch_iface(const DevTables& t, const double* betaR, const double* betaL,
                        double* xsep, int64_t N, hipStream_t s) {
    if (t.P < 2 || N == 0) return hipSuccess;
    const int32_t nsep = t.P - 1;
    int32_t per = (nsep + kScanMaxGroups - 1) / kScanMaxGroups;
    if (per < 4) per = 4;
    const int32_t G = (nsep + per - 1) / per;
    hipLaunchKernelGGL(k_iface, dim3((unsigned)((N + kScanRhs - 1) / kScanRhs)),
                       dim3(kScanRhs * G), 0, s, N, t.P, per, t.rho, t.lam, betaR, betaL, xsep);
    return hipGetLastError();
}

template <int TMAX, typename Fin, typename Xout, int KIND>
static void go_reg(const DevTables& t, const void* F, void* X, int64_t N, int passes,
                   const double* xsep, hipStream_t s) {
    hipLaunchKernelGGL((k_sweep_reg<TMAX, Fin, Xout, KIND>), grid2(N, t.P), dim3(kWG), 0, s,
                       (const Fin*)F, (Xout*)X, N, t.P, t.starts, t.a64, t.b64, t.cp64, t.rd64,
                       t.in64, t.u, t.v, t.a32, t.cp32, t.rd32, t.in32, xsep, passes);
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
