// HIP kernels for gfx950 (MI355X): the per-right-hand-side steps of the
// parallel sweep method.
//
// Mapping: one lane = one right-hand side (the series index n), one
// workgroup = one block j of rows x 256 consecutive right-hand sides.  With
// the RHS-interleaved layout F[i*N + n], every row access of a wavefront is
// one contiguous 256 B (FP32) or 512 B (FP64) span: loads and stores
// coalesce without any transposition.  The coefficients of the constant
// matrix are the same for every lane; they are read through the constant
// address space with wave-uniform addresses, i.e. as scalar loads into
// SGPRs through the scalar cache, which broadcast to the wavefront without
// occupying VGPRs.  (Reading them as constant memory also keeps them scalar
// when their pointers come from a descriptor table, as in the batch.)
//
//   beta   eq. beta_symn: beta^R_j, beta^L_j of block j (FP64 accumulation;
//          rows are read two right-hand sides per lane, 8- or 16-byte
//          loads).
//   iface  Theorem 2 (eq. theor_2): x at the interface rows, in one of three
//          orders: the two first-order recurrences S^R_{k+1} = rho_k S^R_k +
//          beta^R_k and S^L_k = beta^L_k + lam_k S^L_{k+1}, x(s_k) = S^R_k +
//          S^L_k (default); Algorithm 4's dichotomy, level by level; or the
//          double sum itself as one dense product on the FP64 matrix cores.
//   sweep  Lemma 1 / Algorithm 1 step 3: the sweep inside each block with
//          both boundary values known; X leaves with streaming stores.  The
//          sweeps with FP64 results take 35..64-row blocks in two halves on
//          separate wavefronts, joined at the middle row.
//
// Each step is a device function over one work item; the single-matrix
// kernels index items by their 2-D grid, the batch kernels (many matrices of
// uneven sizes in one launch per step) find their matrix and item in a
// descriptor table, in an XCD-aware item order.
#include <type_traits>

#include <hip/hip_ext.h>

#include "tdsolve.h"
#include "tds_internal.h"

namespace tds {

enum SweepKind { kSweep64 = 0, kSweepRefined = 1, kSweep32 = 2 };

// read-only table access through the constant address space (scalar loads)
template <typename T>
using cptr = __attribute__((address_space(4))) const T*;
template <typename T>
__device__ __forceinline__ cptr<T> cst(const T* p) {
    return (cptr<T>)p;
}

// element at a wave-uniform base plus an unsigned 32-bit byte offset: the
// form of the global scalar-base address mode (64-bit base in SGPRs, 32-bit
// offset in one VGPR), which saves a 64-bit VGPR address per row
template <typename T>
__device__ __forceinline__ T& at_off(T* base, uint32_t byte_off) {
    return *(T*)((char*)base + byte_off);
}
template <typename T>
__device__ __forceinline__ const T& at_off(const T* base, uint32_t byte_off) {
    return *(const T*)((const char*)base + byte_off);
}

// Final store of a solution value.  X is written once per solve and not
// read again by it; the non-temporal hint streams it out instead of leaving
// dirty lines that the next reads of F (this solve's or the next one's)
// would have to evict first (measured on the 4096 x 4096 Poisson series:
// 73.5 -> 66.8 us per solve, the beta pass 16.0 -> 12.1 us).
template <typename T>
__device__ __forceinline__ void store_x(T* p, T v) {
    __builtin_nontemporal_store(v, p);
}

// Work-area values (beta weights, interface values) that workgroups of one
// launch hand to each other (the fused order, k_fused) are written through
// to, and read back from, the device-wide coherence point: agent-scope
// relaxed atomic accesses, which gfx950 issues as global stores and loads
// with the sc1 bit.  Each XCD's L2 is not coherent with the other XCDs', so
// ordinary accesses could leave a value in one L2 or read a stale line from
// another.  COH = false: ordinary accesses (values handed over between
// launches, where the kernel boundary makes them visible).
template <bool COH>
__device__ __forceinline__ double ld_w(const double* p) {
    if constexpr (COH)
        return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *p;
}
template <bool COH>
__device__ __forceinline__ void st_w(double* p, double v) {
    if constexpr (COH)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

// ==========================================================================
// beta weights (eq. beta_symn).  Item (tile, j): block j of rows x 64
// consecutive right-hand sides (one per lane); the four wavefronts of the
// workgroup take one quarter of the block's rows each, so every wavefront
// keeps only a quarter of the rows in flight and the grid holds four times
// as many wavefronts as one wavefront per 64 right-hand sides would.  All
// rows of a quarter are loaded before any arithmetic (one round trip to
// memory); rows past the block re-read its last row and get weight zero from
// the zero-padded per-block weight table.  The four partial sums meet in LDS
// and are added in a fixed order (results do not depend on timing).
constexpr int kBetaRhs = 64;
constexpr int kBetaWaves = kWG / kBetaRhs;

template <int TMAX, typename Fin>
__device__ __forceinline__ void beta_item(const DevTables& T, const Fin* __restrict__ F,
                                          int64_t N, int32_t j, int64_t tile,
                                          double* __restrict__ betaR,
                                          double* __restrict__ betaL,
                                          double2* __restrict__ red) {
    const int64_t n0 = tile * kBetaRhs;
    if (n0 >= N) return;                                  // uniform per workgroup
    const int64_t lo = cst(T.starts)[j];
    const int t = (int)(cst(T.starts)[j + 1] - lo);
    const int lane = threadIdx.x % kBetaRhs;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kBetaRhs);
    const bool live = n0 + lane < N;
    // wave-uniform row bases plus one 32-bit byte offset per lane (lanes past
    // N read column N-1 and store nothing)
    const uint32_t off = (uint32_t)(live ? lane : N - 1 - n0) * sizeof(Fin);
    const Fin* fb = F + lo * N + n0;
    double bR = 0.0, bL = 0.0;
    if constexpr (TMAX > 0) {
        constexpr int TQ = TMAX / kBetaWaves;
        const int r0 = wv * TQ;
        const cptr<double2> w = cst(T.wpad + (int64_t)j * TMAX + r0);
        Fin v[TQ];
#pragma unroll
        for (int r = 0; r < TQ; ++r) {
            const int row = r0 + r < t ? r0 + r : t - 1;
            v[r] = at_off(fb + (int64_t)row * N, off);
        }
#pragma unroll
        for (int r = 0; r < TQ; ++r) {
            const double cR = w[r].x, cL = w[r].y;
            bR = fma(cR, (double)v[r], bR);
            bL = fma(cL, (double)v[r], bL);
        }
    } else {
        const int q = (t + kBetaWaves - 1) / kBetaWaves;
        const int r0 = wv * q, r1 = r0 + q < t ? r0 + q : t;
        const cptr<double> gR = cst(T.wR + lo);
        const cptr<double> gL = cst(T.wL + lo);
        constexpr int U = 16;
        int r = r0;
        for (; r + U <= r1; r += U) {
            Fin v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = at_off(fb + (int64_t)(r + u) * N, off);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                bR = fma(gR[r + u], (double)v[u], bR);
                bL = fma(gL[r + u], (double)v[u], bL);
            }
        }
        for (; r < r1; ++r) {
            const double v = (double)at_off(fb + (int64_t)r * N, off);
            bR = fma(gR[r], v, bR);
            bL = fma(gL[r], v, bL);
        }
    }
    if (wv > 0) red[(wv - 1) * kBetaRhs + lane] = make_double2(bR, bL);
    __syncthreads();
    if (wv == 0 && live) {
#pragma unroll
        for (int k = 0; k < kBetaWaves - 1; ++k) {
            const double2 p = red[k * kBetaRhs + lane];
            bR += p.x;
            bL += p.y;
        }
        if (j < T.P - 1) betaR[(int64_t)j * N + n0 + lane] = bR;
        if (j > 0) betaL[(int64_t)j * N + n0 + lane] = bL;
    }
}

// beta_item with V = 2 right-hand sides per lane read by one load per row
// (8 bytes on FP32 input, 16 on FP64), N a multiple of 2 and F aligned to
// the load: half the load instructions, and tiles of 128 right-hand sides,
// the halves sweep's own tiles.  Four right-hand sides per lane (16-byte
// loads, 256-RHS tiles) on FP32 input made the ADI lines' beta pass 54 us
// against 50 us: twice the work per workgroup over half the workgroups.
// Per right-hand side the arithmetic is beta_item's (the same rows per
// wavefront in the same order, the same reduction), so the weights are
// bitwise the same.  Item (tile, j): block j x 64 V right-hand sides.
template <typename Fin>
struct Vec16;                  // the load of V right-hand sides of Fin
template <>
struct Vec16<float> {
    static constexpr int V = 2;
    using type = float2;
};
template <>
struct Vec16<double> {
    static constexpr int V = 2;
    using type = double2;
};

template <int TMAX, typename Fin, bool COH = false>
__device__ __forceinline__ void beta_item_vec(const DevTables& T, const Fin* __restrict__ F,
                                              int64_t N, int32_t j, int64_t tile,
                                              double* __restrict__ betaR,
                                              double* __restrict__ betaL,
                                              double2* __restrict__ red) {
    constexpr int TQ = TMAX / kBetaWaves;
    constexpr int V = Vec16<Fin>::V;
    using VT = typename Vec16<Fin>::type;
    const int64_t n0 = tile * (V * kBetaRhs);
    if (n0 >= N) return;                                  // uniform per workgroup
    const int64_t lo = cst(T.starts)[j];
    const int t = (int)(cst(T.starts)[j + 1] - lo);
    const int lane = threadIdx.x % kBetaRhs;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kBetaRhs);
    const bool live = n0 + V * lane < N;
    // lanes past N read the last group of V columns and store nothing
    const uint32_t off = (uint32_t)(live ? V * lane : N - V - n0) * sizeof(Fin);
    const Fin* fb = F + lo * N + n0;
    const int r0 = wv * TQ;
    const cptr<double2> w = cst(T.wpad + (int64_t)j * TMAX + r0);
    VT v[TQ];
#pragma unroll
    for (int r = 0; r < TQ; ++r) {
        const int row = r0 + r < t ? r0 + r : t - 1;
        v[r] = at_off((const VT*)(fb + (int64_t)row * N), off);
    }
    double bR[V], bL[V];
#pragma unroll
    for (int q = 0; q < V; ++q) bR[q] = bL[q] = 0.0;
#pragma unroll
    for (int r = 0; r < TQ; ++r) {
        const double cR = w[r].x, cL = w[r].y;
        Fin e[V];
        __builtin_memcpy(e, &v[r], sizeof(VT));
#pragma unroll
        for (int q = 0; q < V; ++q) {
            bR[q] = fma(cR, (double)e[q], bR[q]);
            bL[q] = fma(cL, (double)e[q], bL[q]);
        }
    }
    if (wv > 0)
#pragma unroll
        for (int q = 0; q < V; ++q)
            red[((wv - 1) * V + q) * kBetaRhs + lane] = make_double2(bR[q], bL[q]);
    __syncthreads();
    if (wv == 0 && live) {
#pragma unroll
        for (int q = 0; q < V; ++q)
#pragma unroll
            for (int k = 0; k < kBetaWaves - 1; ++k) {
                const double2 p = red[(k * V + q) * kBetaRhs + lane];
                bR[q] += p.x;
                bL[q] += p.y;
            }
        double* oR = &betaR[(int64_t)j * N + n0 + V * lane];
        double* oL = &betaL[(int64_t)j * N + n0 + V * lane];
#pragma unroll
        for (int q = 0; q < V; ++q) {
            if (j < T.P - 1) st_w<COH>(&oR[q], bR[q]);
            if (j > 0) st_w<COH>(&oL[q], bL[q]);
        }
    }
}

// Batch beta weights: one workgroup per item (block j x 256 right-hand
// sides), each wavefront 64 right-hand sides and every row of the block.
// The batch's blocks are short (<= TMAX = 32 or 64 rows), so beta_item's
// split of the rows over the four wavefronts would leave a workgroup about
// 8 KB of input; here a workgroup carries four times that, with a quarter
// of the launches and no LDS reduction.  Each wavefront forms the four
// quarter sums of beta_item separately and adds them in the order of its
// reduction, so the weights are bitwise those of a single-matrix plan.
template <int TMAX, typename Fin, bool COH = false>
__device__ __forceinline__ void beta_rows_item(const DevTables& T, const Fin* __restrict__ F,
                                               int64_t N, int32_t j, int64_t n0,
                                               double* __restrict__ betaR,
                                               double* __restrict__ betaL) {
    if (n0 >= N) return;                                  // uniform per wavefront
    const int64_t lo = cst(T.starts)[j];
    const int t = (int)(cst(T.starts)[j + 1] - lo);
    const int lane = threadIdx.x % kBetaRhs;
    const bool live = n0 + lane < N;
    const uint32_t off = (uint32_t)(live ? lane : N - 1 - n0) * sizeof(Fin);
    const Fin* fb = F + lo * N + n0;
    constexpr int TQ = TMAX / kBetaWaves;
    const cptr<double2> w = cst(T.wpad + (int64_t)j * TMAX);
    Fin v[TMAX];
#pragma unroll
    for (int r = 0; r < TMAX; ++r) v[r] = at_off(fb + (int64_t)(r < t ? r : t - 1) * N, off);
    double bR = 0.0, bL = 0.0;
#pragma unroll
    for (int q = 0; q < kBetaWaves; ++q) {
        double qR = 0.0, qL = 0.0;
#pragma unroll
        for (int r = 0; r < TQ; ++r) {
            const double cR = w[q * TQ + r].x, cL = w[q * TQ + r].y;
            qR = fma(cR, (double)v[q * TQ + r], qR);
            qL = fma(cL, (double)v[q * TQ + r], qL);
        }
        if (q == 0) {
            bR = qR;
            bL = qL;
        } else {
            bR += qR;
            bL += qL;
        }
    }
    if (!live) return;
    if (j < T.P - 1) st_w<COH>(&betaR[(int64_t)j * N + n0 + lane], bR);
    if (j > 0) st_w<COH>(&betaL[(int64_t)j * N + n0 + lane], bL);
}

// ==========================================================================
// Interface step (Theorem 2): the O(P) recurrences
//   forward   y_j = rho_j y_{j-1} + beta^R_j,  j = 0..P-2 (y_{-1} = 0),
//             so that S^R_{j+1} = y_j;
//   backward  z_j = lam_j z_{j+1} + beta^L_j,  j = P-1..1 (z_P = 0),
//             so that S^L_j = z_j;
//   x(s_k) = S^R_k + S^L_k, k = 1..P-1  (xsep row k-1),
// as a two-level scan: workgroup = R right-hand sides x G groups of `per`
// consecutive blocks (single-matrix kernel: R = 16, up to 64 groups; batch
// kernel: G x R = 256 with a shape per matrix, see batch_scan_shape).  Each
// thread loads its group's beta values once, scans them with zero input,
// the group carries (product of the factors, partial value) are combined
// through LDS, then each thread finishes its group with the true input.
// When a thread keeps its beta values in registers (per <= MAXPER: 8 in the
// single-matrix kernel, 16 in the batch kernel), S^R goes to LDS and the
// thread owning the same interface row in the backward direction writes
// S^R + S^L to xsep once; otherwise S^R is written to xsep and S^L added
// after a barrier.
constexpr int kScanMaxGroupsSingle = 64;  // single-matrix workgroups (up to 1024 threads)
constexpr int kScanMaxPer = 8;     // beta values a thread keeps in registers (single)
constexpr int kChainChunk = 8;     // beta values read per memory round trip

// S^R recurrence y <- rho_j y + beta^R_j for j = j0 .. j1-1 (rho_0 is not
// used: S^R_0 = 0), reading kChainChunk values per round trip; every y is
// stored to out[j] when out is given.
template <bool COH = false>
__device__ __forceinline__ double chain_right(double y, const cptr<double> rho,
                                              const double* __restrict__ beta, int64_t N,
                                              int64_t n, int32_t j0, int32_t j1,
                                              double* __restrict__ out) {
    for (int32_t jb = j0; jb < j1; jb += kChainChunk) {
        double v[kChainChunk];
#pragma unroll
        for (int u = 0; u < kChainChunk; ++u)
            v[u] = (jb + u < j1) ? ld_w<COH>(&beta[(int64_t)(jb + u) * N + n]) : 0.0;
#pragma unroll
        for (int u = 0; u < kChainChunk; ++u) {
            const int32_t j = jb + u;
            if (j < j1) {
                y = fma((j > 0) ? rho[j] : 0.0, y, v[u]);
                if (out) st_w<COH>(&out[(int64_t)j * N + n], y);
            }
        }
    }
    return y;
}

// S^L recurrence z <- beta^L_j + lam_j z for j = j1 down to j0+1 (lam_{P-1}
// is not used: S^L_P = 0); with out given, z is added to out[j-1].
template <bool COH = false>
__device__ __forceinline__ double chain_left(double z, const cptr<double> lam, int32_t P,
                                             const double* __restrict__ beta, int64_t N,
                                             int64_t n, int32_t j1, int32_t j0,
                                             double* __restrict__ out) {
    for (int32_t jb = j1; jb > j0; jb -= kChainChunk) {
        double v[kChainChunk];
#pragma unroll
        for (int u = 0; u < kChainChunk; ++u)
            v[u] = (jb - u > j0) ? ld_w<COH>(&beta[(int64_t)(jb - u) * N + n]) : 0.0;
#pragma unroll
        for (int u = 0; u < kChainChunk; ++u) {
            const int32_t j = jb - u;
            if (j > j0) {
                z = fma((j < P - 1) ? lam[j] : 0.0, z, v[u]);
                if (out) {
                    double* o = &out[(int64_t)(j - 1) * N + n];
                    st_w<COH>(o, ld_w<COH>(o) + z);
                }
            }
        }
    }
    return z;
}

// LDS of one interface-scan workgroup (G groups): the group carries
// carry[2][G][kScanRhs], the products of the factors prod[2][G] and, when
// the beta values stay in registers, S^R by interface row sr[G per][kScanRhs].
__host__ __device__ constexpr size_t scan_lds_doubles(int32_t G, int32_t per,
                                                      int32_t maxper = kScanMaxPer,
                                                      int32_t R = kScanRhs) {
    return (size_t)2 * G * R + 2 * G + (per <= maxper ? (size_t)G * per * R : 0);
}

template <int MAXPER, bool COH = false>
__device__ __forceinline__ void iface_item(const DevTables& T, int64_t N, int32_t per,
                                           int32_t G, const double* __restrict__ betaR,
                                           const double* __restrict__ betaL,
                                           double* __restrict__ xsep, int64_t sblk,
                                           double* smem, int lgR) {
    const int32_t P = T.P;
    // R = 2^lgR right-hand sides per group, one lane each
    const int R = 1 << lgR;
    const int lane = threadIdx.x & (R - 1);
    const int g = threadIdx.x >> lgR;
    const int64_t n = (sblk << lgR) + lane;
    const bool grp = g < G;                 // this thread's group exists
    const bool live = (n < N) && grp;
    const cptr<double> rho = cst(T.rho), lam = cst(T.lam);
    // forward group: j in [f0, f1); backward group: j in (b0, b1]
    const int32_t f0 = g * per, f1 = min(f0 + per, P - 1);
    const int32_t b1 = P - 1 - g * per, b0 = max(b1 - per, 0);

    double yl = 0.0, pr = 1.0, zl = 0.0, pl = 1.0;
    double bRv[MAXPER], bLv[MAXPER];
    double rv[MAXPER], lv[MAXPER];     // the group's factors (keep path)
    const bool keep = per <= MAXPER;
    if (grp) {
        // the products of the factors do not depend on the right-hand side;
        // on the keep path every factor is loaded at once (one round trip)
        // and kept for the recurrences
        if (keep) {
#pragma unroll
            for (int u = 0; u < MAXPER; ++u) {
                const int32_t jf = f0 + u, jb = b1 - u;
                rv[u] = (jf < f1 && jf > 0) ? rho[jf] : 0.0;
                lv[u] = (jb > b0 && jb < P - 1) ? lam[jb] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < MAXPER; ++u) {
                if (f0 + u < f1) pr *= rv[u];
                if (b1 - u > b0) pl *= lv[u];
            }
        } else {
            for (int32_t j = f0; j < f1; ++j) pr *= (j > 0) ? rho[j] : 0.0;
            for (int32_t j = b1; j > b0; --j) pl *= (j < P - 1) ? lam[j] : 0.0;
        }
    }
    if (live) {
        if (keep) {
#pragma unroll
            for (int u = 0; u < MAXPER; ++u) {
                const int32_t jf = f0 + u, jb = b1 - u;
                bRv[u] = (jf < f1) ? ld_w<COH>(&betaR[(int64_t)jf * N + n]) : 0.0;
                bLv[u] = (jb > b0) ? ld_w<COH>(&betaL[(int64_t)jb * N + n]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < MAXPER; ++u) {
                const int32_t jf = f0 + u, jb = b1 - u;
                if (jf < f1) yl = fma(rv[u], yl, bRv[u]);
                if (jb > b0) zl = fma(lv[u], zl, bLv[u]);
            }
        } else {
            yl = chain_right<COH>(yl, rho, betaR, N, n, f0, f1, nullptr);
            zl = chain_left<COH>(zl, lam, P, betaL, N, n, b1, b0, nullptr);
        }
    }
    double* carry = smem;                              // [2][G][R]
    double* prod = smem + 2 * G * R;            // [2][G]
    double* sr = prod + 2 * G;                          // [G per][R]
    if (grp) {
        carry[g * R + lane] = yl;
        carry[(G + g) * R + lane] = zl;
        if (lane == 0) {
            prod[g] = pr;
            prod[G + g] = pl;
        }
    }
    __syncthreads();
    double yin = 0.0, zin = 0.0;
    {
        // the carries of the groups before this one, in group order; LDS
        // reads four groups at a time, so that one wait covers four steps
        const int ng = g < G ? g : G;
        int q = 0;
        for (; q + 4 <= ng; q += 4) {
            double py[4], cy[4], pz[4], cz[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                py[u] = prod[q + u];
                cy[u] = carry[(q + u) * R + lane];
                pz[u] = prod[G + q + u];
                cz[u] = carry[(G + q + u) * R + lane];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                yin = fma(py[u], yin, cy[u]);
                zin = fma(pz[u], zin, cz[u]);
            }
        }
        for (; q < ng; ++q) {
            yin = fma(prod[q], yin, carry[q * R + lane]);
            zin = fma(prod[G + q], zin, carry[(G + q) * R + lane]);
        }
    }
    // finish the forward group: y_j = S^R_{j+1} into LDS or xsep
    if (live) {
        double y = yin;
        if (keep) {
#pragma unroll
            for (int u = 0; u < MAXPER; ++u) {
                const int32_t j = f0 + u;
                if (j < f1) {
                    y = fma(rv[u], y, bRv[u]);
                    sr[j * R + lane] = y;
                }
            }
        } else {
            chain_right<COH>(y, rho, betaR, N, n, f0, f1, xsep);
        }
    }
    __syncthreads();     // S^R of every group is in LDS or xsep (same workgroup)
    if (!live) return;
    double z = zin;
    if (keep) {
#pragma unroll
        for (int u = 0; u < MAXPER; ++u) {
            const int32_t j = b1 - u;
            if (j > b0) {
                z = fma(lv[u], z, bLv[u]);
                st_w<COH>(&xsep[(int64_t)(j - 1) * N + n], sr[(j - 1) * R + lane] + z);   // S^R_j + S^L_j
            }
        }
    } else {
        chain_left<COH>(z, lam, P, betaL, N, n, b1, b0, xsep);   // x(s_j) = S^R_j + S^L_j
    }
}

// ==========================================================================
// Interface step by the dichotomy (Algorithm 4 step 2.2, Theorem 3,
// eq. omega_i).  The p = P-1 interface rows are found level by level:
// level l = 1 .. floor(log2 p) + 1 takes the rows i = step (2m + 1) <= p,
// step = 2^(levels - l); the nearest interface rows already known are
// k1 = i - step (0: the left end of the domain) and k2 = i + step (P, the
// right end, when past p).  Between them the two partial sums continue from
// the known ones (the reading of Theorem 3's correction terms):
//     S^R_i from S^R_{k1} by S^R_{j+1} = rho_j S^R_j + beta^R_j, j = k1..i-1,
//     S^L_i from S^L_{k2} by S^L_j = beta^L_j + lam_j S^L_{j+1}, j = k2-1..i,
// and x(s_i) = S^R_i + S^L_i.  Rows of one level are independent (the
// remark after Algorithm 4): they are spread over the workgroup's four row
// slots, its 64 lanes being 64 right-hand sides, and the levels are
// separated by workgroup barriers.  S^R and S^L are kept in work arrays of
// (P + 1) x N each.  The same values as the recurrences of k_iface up to
// rounding; O(P log P) work per right-hand side instead of O(P).
constexpr int kDichRhs = 64;
constexpr int kDichSlots = kWG / kDichRhs;

__global__ __launch_bounds__(kWG) void k_iface_dich(DevTables T, int64_t N,
                                                   const double* __restrict__ betaR,
                                                   const double* __restrict__ betaL,
                                                   double* SR, double* SL,
                                                   double* __restrict__ xsep) {
    const int32_t P = T.P;
    const int32_t p = P - 1;
    const int lane = threadIdx.x % kDichRhs;
    const int slot = __builtin_amdgcn_readfirstlane(threadIdx.x / kDichRhs);
    const int64_t n = (int64_t)blockIdx.x * kDichRhs + lane;
    const bool live = n < N;
    const cptr<double> rho = cst(T.rho), lam = cst(T.lam);
    int levels = 0;
    while ((int64_t(1) << levels) <= p) ++levels;          // floor(log2 p) + 1
    for (int l = 1; l <= levels; ++l) {
        const int32_t step = 1 << (levels - l);
        for (int32_t m = slot;; m += kDichSlots) {
            const int32_t i = step * (2 * m + 1);
            if (i > p) break;
            if (!live) continue;
            const int32_t k1 = i - step, k2 = (i + step <= p) ? i + step : P;
            double sr = (k1 == 0) ? 0.0 : SR[(int64_t)k1 * N + n];
            sr = chain_right(sr, rho, betaR, N, n, k1, i, nullptr);
            double sl = (k2 == P) ? 0.0 : SL[(int64_t)k2 * N + n];
            sl = chain_left(sl, lam, P, betaL, N, n, k2 - 1, i - 1, nullptr);
            SR[(int64_t)i * N + n] = sr;
            SL[(int64_t)i * N + n] = sl;
        }
        __syncthreads();        // this level's sums are the next level's k1, k2
    }
    if (!live) return;
    for (int32_t k = 1 + slot; k <= p; k += kDichSlots)
        xsep[(int64_t)(k - 1) * N + n] = SR[(int64_t)k * N + n] + SL[(int64_t)k * N + n];
}

// ==========================================================================
// Interface values by Theorem 2's double sum (eq. theor_2) as one dense
// product on the FP64 matrix cores:
//     Xsep[k-1][n] = sum_j KR[k][j] beta^R_j[n] + sum_j KL[k][j] beta^L_j[n],
// k = 1..P-1, with the ratio products KR[k][j] = rho_{j+1} ... rho_{k-1}
// (j < k) and KL[k][j] = lam_k ... lam_{j-1} (j >= k) from the preliminary
// step.  The coefficient table is k-major, Kt[kk][r] (output row r = k-1,
// combined index kk = j for the right part, Pc + j for the left part;
// Pc = P rounded up to 4, rows padded to Mr, a multiple of 64, zeros
// elsewhere).
//
// Workgroup: 16 right-hand sides x 64 output rows, one wavefront per 16-row
// tile.  A wavefront only visits the k-steps (4 values of j each) whose
// coefficients are not all zero for its rows r = k-1: the right part up to
// j = its last row (KR vanishes for j >= k), the left part from the step
// holding its first k (KL vanishes for j < k).  It loads the operands of up
// to 32 steps into registers at once (coefficients from the small table,
// which stays in L2; beta values straight from memory), then chains the
// steps' V_MFMA_F64_16X16X4F64 on one accumulator.  Operand layout of that
// instruction (wave64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and receives D[4 i + l / 16][l % 16] in element i (rows
// interleaved across the four lane groups; checked by a probe on gfx950).
constexpr int kDenseCols = 16;      // right-hand sides per workgroup
constexpr int kDenseRows = 64;      // output rows per workgroup (4 tiles)
constexpr int kDenseBatch = 32;     // k-steps whose operands are loaded together

// one workgroup's share of the dense product: output rows by * kDenseRows
// .. + 63 (one 16-row tile per wavefront) x right-hand sides bx *
// kDenseCols .. + 15; BATCH k-steps have their operands loaded at once
template <int BATCH, bool COH = false>
__device__ __forceinline__ void dense_item(const double* __restrict__ Kt, int32_t Pc, int32_t Mr,
                                           int32_t P, int64_t N, const double* __restrict__ betaR,
                                           const double* __restrict__ betaL,
                                           double* __restrict__ xsep, int64_t bx, int32_t by) {
    using d4 = __attribute__((ext_vector_type(4))) double;
    const int lane = threadIdx.x % 64;
    const int tile = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int col = lane % 16, kq = lane / 16;
    const int64_t n = bx * kDenseCols + col;
    const int32_t rlo = by * kDenseRows + 16 * tile;
    if (rlo >= P - 1) return;                      // tile past the last interface row
    const int32_t rhi = min(rlo + 15, P - 2);
    // steps: right part j4 = 0, 4, .., <= rhi; left part j4 = (rlo + 1) & ~3, .., <= P-1
    const int32_t nR = rhi / 4 + 1;
    const int32_t jl0 = (rlo + 1) & ~3;
    const int32_t nL = (P - 1 - jl0) / 4 + 1;
    const int32_t steps = nR + nL;
    const bool live = n < N;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int32_t s0 = 0; s0 < steps; s0 += BATCH) {
        double av[BATCH], bv[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int32_t st = s0 + u;
            const bool left = st >= nR;
            const int32_t j = left ? jl0 + 4 * (st - nR) + kq : 4 * st + kq;
            const int32_t kk = left ? Pc + j : j;
            const bool ok = st < steps && j < P;
            // the step's four j can reach past the weights this tile uses
            // (beta^R_j for j <= rhi, beta^L_j for j > rlo); those rows of
            // the work area (beta^R_{P-1}, beta^L_0 among them) are never
            // written, so they are not read either: their coefficients are
            // zero, but 0 times a stale non-finite value is not
            const bool need = left ? (j > rlo) : (j <= rhi);
            av[u] = ok ? Kt[(int64_t)kk * Mr + rlo + col] : 0.0;
            bv[u] = (ok && live && need) ? ld_w<COH>(&(left ? betaL : betaR)[(int64_t)j * N + n]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u)
            if (s0 + u < steps) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    if (!live) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int32_t r = rlo + 4 * i + kq;
        if (r < P - 1) st_w<COH>(&xsep[(int64_t)r * N + n], acc[i]);
    }
}

__global__ __launch_bounds__(kWG) void k_iface_dense(const double* __restrict__ Kt, int32_t Pc,
                                                     int32_t Mr, int32_t P, int64_t N,
                                                     const double* __restrict__ betaR,
                                                     const double* __restrict__ betaL,
                                                     double* __restrict__ xsep) {
    dense_item<kDenseBatch>(Kt, Pc, Mr, P, N, betaR, betaL, xsep, (int64_t)blockIdx.x,
                            (int32_t)blockIdx.y);
}

// ==========================================================================
// Block sweep, register-resident.  Block j's interior rows i0..i1 (block 0
// starts at row 0; the others at the row after their left interface row)
// are solved with x at the interface rows s_j (left, xl) and s_{j+1}
// (right, xr) known (Lemma 1).  Each lane keeps its whole column of the
// block in VGPRs: F is read once and X written once.  The tables are
// separate arrays so that each sweep fetches only the bytes it uses (the
// scalar fetch volume per row shows directly in the run time).
//
// One body serves every block length cnt <= TMAX: rows cnt..TMAX-1 are
// "phantom" rows.  They re-read the block's last real row of F and the
// (padded, always in-bounds) table rows that follow, so their values stay
// finite, and they never feed back into real rows because the last real
// row's elimination factor and block-interior coupling are zero.  They are
// not stored.
// the block's interior rows of F for one lane (rows past cnt re-read the
// last row)
// (fb: wave-uniform base of the block's first interior row, lane: the
// lane's offset; the loads then take the scalar-base addressing form)
template <int TMAX, typename Fin>
__device__ __forceinline__ void sweep_load(const Fin* __restrict__ fb, int lane, int64_t N,
                                           int cnt, Fin (&f)[TMAX]) {
#pragma unroll
    for (int r = 0; r < TMAX; ++r) f[r] = (fb + (int64_t)(r < cnt ? r : cnt - 1) * N)[lane];
}

// Zero-boundary solve of one block (or half block) of the refined sweep:
// x0 = T^{-1} f by an FP32 sweep, then `passes` times FP64 residual -> FP32
// sweep of the residual -> FP64 update.  T's tables are read from row i0;
// my_f holds the lane's FP32 right-hand side in LDS (row r at
// my_f[r * STRIDE], STRIDE = the workgroup's lanes).
template <int TMAX, bool GEN, int STRIDE = kWG>
__device__ __forceinline__ void refined_solve(const DevTables& T, int64_t i0,
                                              const float* __restrict__ my_f, int passes,
                                              double (&x)[TMAX]) {
    const cptr<double> b64 = cst(T.b64 + i0);
    const cptr<float> cp32 = cst(T.cp32 + i0), rd32 = cst(T.rd32 + i0);
    const cptr<float> inl32 = cst((GEN ? T.inl32 : T.in32) + i0);
    float w[TMAX];
#pragma unroll
    for (int r = 0; r < TMAX; ++r) {
        if ((r & 3) == 0) __builtin_amdgcn_sched_barrier(0);
        const float prev = (r > 0) ? w[r - 1] : 0.0f;
        const float sub = (r > 0) ? inl32[r - 1] : 0.0f;
        w[r] = (my_f[r * STRIDE] - sub * prev) * rd32[r];
    }
    {
        float xs = 0.0f;
#pragma unroll
        for (int r = TMAX - 1; r >= 0; --r) {
            if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            xs = w[r] - cp32[r] * xs;
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
        const cptr<double> in64p = cst(T.in64 + i0) + z;
        const cptr<double> inl64p = GEN ? cst(T.inl64 + i0) + z : in64p;
        const cptr<double> b64p = b64 + z;
        const cptr<float> inl32p = inl32 + z, cp32p = cp32 + z, rd32p = rd32 + z;
#pragma unroll
        for (int r = 0; r < TMAX; ++r) {
            // bound the scheduler's look-ahead: the residuals do not
            // depend on the elimination chain, and computing them all
            // ahead of it would hold 64 FP64 values in registers
            if ((r & 3) == 0) __builtin_amdgcn_sched_barrier(0);
            double res = (double)my_f[r * STRIDE] - b64p[r] * x[r];
            if (r > 0) res -= inl64p[r - 1] * x[r - 1];
            if (r + 1 < TMAX) res -= in64p[r] * x[r + 1];
            const float prev = (r > 0) ? w[r - 1] : 0.0f;
            const float sub = (r > 0) ? inl32p[r - 1] : 0.0f;
            w[r] = ((float)res - sub * prev) * rd32p[r];
        }
        float dl = 0.0f;
#pragma unroll
        for (int r = TMAX - 1; r >= 0; --r) {
            if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            dl = w[r] - cp32p[r] * dl;
            x[r] += (double)dl;
        }
    }
}

// The last residual pass of the refined sweep, over a block (or half
// block) of cnt rows whose boundary values are known: xL beside its first
// row (coupling cl) and xR beside row cnt-1 (coupling cr); x holds the
// block's values including the boundary responses.  The residual is formed
// in FP64 with the boundary terms and eliminated in FP32 as in the other
// passes (boundary_elim), and the back substitution carries each row's
// rounded update into the next row in FP64 (carried_back_sub):
//     y_r = x_r + (w_r - cp_r (y_{r+1} - x_{r+1})),
// so the result is the solution of the bidiagonal system U y = U x + w up
// to one rounding per row, as in a direct sweep: its rounding errors stay
// correlated along the block instead of adding an independent error to
// every row (which would raise the residual by about the ratio of |A| to
// the elimination's lower factor).
template <int TMAX, bool GEN, int STRIDE = kWG>
__device__ __forceinline__ void boundary_elim(const DevTables& T, int64_t i0,
                                              const float* __restrict__ my_f, int cnt, double cl,
                                              double xL, double cr, double xR,
                                              const double (&x)[TMAX], float (&w)[TMAX]) {
    asm volatile("" ::: "memory");
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    const cptr<double> in64p = cst(T.in64 + i0) + z;
    const cptr<double> inl64p = GEN ? cst(T.inl64 + i0) + z : in64p;
    const cptr<double> b64p = cst(T.b64 + i0) + z;
    const cptr<float> inl32p = cst((GEN ? T.inl32 : T.in32) + i0) + z;
    const cptr<float> rd32p = cst(T.rd32 + i0) + z;
#pragma unroll
    for (int r = 0; r < TMAX; ++r) {
        if ((r & 3) == 0) __builtin_amdgcn_sched_barrier(0);
        double res = (double)my_f[r * STRIDE] - b64p[r] * x[r];
        if (r > 0) res -= inl64p[r - 1] * x[r - 1];
        if (r + 1 < TMAX) res -= in64p[r] * x[r + 1];
        if (r == 0) res -= cl * xL;
        // the right boundary's row: a scalar select of the coupling, not a
        // per-lane select of the residual
        res = fma(-((r == cnt - 1) ? cr : 0.0), xR, res);
        const float prev = (r > 0) ? w[r - 1] : 0.0f;
        const float sub = (r > 0) ? inl32p[r - 1] : 0.0f;
        w[r] = ((float)res - sub * prev) * rd32p[r];
    }
}

// carry: the update beyond the last row (zero, or a correction of the value
// there, entering the last row through coupling c_last)
template <int TMAX>
__device__ __forceinline__ void carried_back_sub(const DevTables& T, int64_t i0,
                                                 const float (&w)[TMAX], double carry,
                                                 double c_last, double (&x)[TMAX]) {
    asm volatile("" ::: "memory");
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    const cptr<float> cp32p = cst(T.cp32 + i0) + z;
#pragma unroll
    for (int r = TMAX - 1; r >= 0; --r) {
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        // converted here, not beside the elimination (which would hold
        // every row's w in FP64)
        float wr = w[r];
        asm volatile("" : "+v"(wr));
        const double cp = (r == TMAX - 1) ? c_last : (double)cp32p[r];
        const double y = x[r] + fma(-cp, carry, (double)wr);
        carry = y - x[r];
        x[r] = y;
    }
}

template <int TMAX, bool GEN, int STRIDE = kWG>
__device__ __forceinline__ void refined_boundary_pass(const DevTables& T, int64_t i0,
                                                      const float* __restrict__ my_f, int cnt,
                                                      double cl, double xL, double cr, double xR,
                                                      double (&x)[TMAX]) {
    float w[TMAX];
    boundary_elim<TMAX, GEN, STRIDE>(T, i0, my_f, cnt, cl, xL, cr, xR, x, w);
    carried_back_sub<TMAX>(T, i0, w, 0.0, 0.0, x);
}

template <int TMAX, typename Fin, typename Xout, int KIND, bool GEN>
__device__ __forceinline__ void sweep_body(const Fin (&f)[TMAX], Xout* __restrict__ xb, int lane,
                                           int64_t N, int cnt, double cl, double xl, double cr,
                                           double xr, const DevTables& T, int64_t i0,
                                           float* __restrict__ my_f, int passes) {
    // sub-diagonal: its own table for a non-symmetric A, else the one
    // off-diagonal table (one scalar stream fewer per row)
    const cptr<double> l64 = cst((GEN ? T.l64 : T.a64) + i0);
    const cptr<double> cp64 = cst(T.cp64 + i0), rd64 = cst(T.rd64 + i0);
    const cptr<double> uu = cst(T.u + i0), vv = cst(T.v + i0);
    const cptr<float> l32 = cst((GEN ? T.l32 : T.a32) + i0), cp32 = cst(T.cp32 + i0),
                      rd32 = cst(T.rd32 + i0);

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
                const double sub = (r > 0) ? l64[r - 1] : 0.0;
                d[r] = (g(r) - sub * prev) * rd64[r];
            }
            double x = 0.0;
#pragma unroll
            for (int r = TMAX - 1; r >= 0; --r) {
                x = d[r] - cp64[r] * x;
                if (r < cnt) store_x(&(xb + (int64_t)r * N)[lane], (Xout)x);
            }
        } else {
            float w[TMAX];
#pragma unroll
            for (int r = 0; r < TMAX; ++r) {
                const float prev = (r > 0) ? w[r - 1] : 0.0f;
                const float sub = (r > 0) ? l32[r - 1] : 0.0f;
                w[r] = ((float)g(r) - sub * prev) * rd32[r];
            }
            float x = 0.0f;
#pragma unroll
            for (int r = TMAX - 1; r >= 0; --r) {
                x = w[r] - cp32[r] * x;
                if (r < cnt) store_x(&(xb + (int64_t)r * N)[lane], (Xout)x);
            }
        }
    } else {
        // Refined: the block is solved with zero boundary values, x0 =
        // T^{-1} f (refined_solve); the interface values enter at the end by
        // superposition, x = x0 + xl u + xr v.  (With the boundary terms
        // inside the right-hand side every pass would carry a row-dependent
        // condition.)
#pragma unroll
        for (int r = 0; r < TMAX; ++r) my_f[r * kWG] = (float)f[r];
        double x[TMAX];
        // after the zero-boundary passes, one more over the whole solution
        // with its boundary values (refined_boundary_pass)
        refined_solve<TMAX, GEN>(T, i0, my_f, passes, x);
#pragma unroll
        for (int r = 0; r < TMAX; ++r) x[r] = fma(xr, vv[r], fma(xl, uu[r], x[r]));
        if (passes >= 1) refined_boundary_pass<TMAX, GEN>(T, i0, my_f, cnt, cl, xl, cr, xr, x);
#pragma unroll
        for (int r = 0; r < TMAX; ++r)
            if (r < cnt) store_x(&(xb + (int64_t)r * N)[lane], (Xout)x[r]);
    }
}

template <int TMAX, typename Fin, typename Xout, int KIND, bool GEN, bool COH = false>
__device__ __forceinline__ void sweep_item(const DevTables& T, const Fin* __restrict__ F,
                                           Xout* __restrict__ X, int64_t N, int32_t j,
                                           int64_t tile, const double* __restrict__ xsep,
                                           int passes, float* s_f) {
    const int32_t P = T.P;
    const int64_t seg_lo = cst(T.starts)[j], seg_hi = cst(T.starts)[j + 1];
    const int64_t i0 = (j == 0) ? seg_lo : seg_lo + 1;
    const int cnt = (int)(seg_hi - i0);
    const int64_t n = tile * kWG + threadIdx.x;
    if (n >= N) return;
    const double xl = (j > 0) ? ld_w<COH>(&xsep[(int64_t)(j - 1) * N + n]) : 0.0;
    const double xr = (j < P - 1) ? ld_w<COH>(&xsep[(int64_t)j * N + n]) : 0.0;
    const double cl = (j > 0) ? cst(GEN ? T.l64 : T.a64)[i0 - 1] : 0.0;   // A[i0][i0-1]
    const double cr = (j < P - 1) ? cst(T.a64)[seg_hi - 1] : 0.0; // A[i1][i1+1]
    if (j > 0) store_x(&X[seg_lo * N + n], (Xout)xl);
    Fin f[TMAX];
    const int lane = threadIdx.x;
    sweep_load<TMAX, Fin>(F + i0 * N + tile * kWG, lane, N, cnt, f);
    sweep_body<TMAX, Fin, Xout, KIND, GEN>(f, X + i0 * N + tile * kWG, lane, N, cnt, cl, xl, cr, xr, T,
                                      i0, s_f + lane, passes);
}

// Block sweep for blocks longer than the register path holds: the forward
// elimination is kept in X itself and read back by the back substitution.
// FP64 arithmetic except for KIND == kSweep32.
template <typename Fin, typename Xout, int KIND, bool GEN>
__device__ __forceinline__ void sweep_stream_item(const DevTables& T, const Fin* __restrict__ F,
                                                  Xout* __restrict__ X, int64_t N, int32_t j,
                                                  int64_t tile, const double* __restrict__ xsep) {
    const int32_t P = T.P;
    const cptr<double> a64 = cst(T.a64), l64 = cst(GEN ? T.l64 : T.a64), cp64 = cst(T.cp64),
                       rd64 = cst(T.rd64);
    const int64_t seg_lo = cst(T.starts)[j], seg_hi = cst(T.starts)[j + 1];
    const int64_t i0 = (j == 0) ? seg_lo : seg_lo + 1;
    const int64_t cnt = seg_hi - i0;
    const int64_t n = tile * kWG + threadIdx.x;
    if (n >= N) return;
    const double xl = (j > 0) ? xsep[(int64_t)(j - 1) * N + n] : 0.0;
    const double xr = (j < P - 1) ? xsep[(int64_t)j * N + n] : 0.0;
    const double cl = (j > 0) ? l64[i0 - 1] : 0.0;
    const double cr = (j < P - 1) ? a64[seg_hi - 1] : 0.0;
    if (j > 0) store_x(&X[seg_lo * N + n], (Xout)xl);
    double prev = 0.0;
    for (int64_t r = 0; r < cnt; ++r) {
        const int64_t i = i0 + r;
        double v = (double)F[i * N + n];
        if (r == 0) v -= cl * xl;
        if (r == cnt - 1) v -= cr * xr;
        const double sub = (r > 0) ? l64[i - 1] : 0.0;
        double d;
        if (KIND == kSweep32)
            d = (double)(((float)v - (float)sub * (float)prev) * (float)rd64[i]);
        else
            d = (v - sub * prev) * rd64[i];
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
        store_x(&X[i * N + n], (Xout)x);
    }
}

// Occupancy target (waves per SIMD) of the refined sweep, which holds about
// 3 registers per row (x in FP64, the FP32 elimination value; F sits in
// LDS): 4 up to 32 rows (the last pass with boundary values needs a few
// more than 128 registers otherwise), 2 up to 64; the other sweeps are left
// to the compiler.
template <int KIND, int TMAX>
constexpr int sweep_min_waves() {
    return TMAX > 64 ? 1 : KIND == kSweepRefined ? (TMAX <= 32 ? 4 : 2) : 1;
}

// ==========================================================================
// single-matrix kernels: grid (RHS tiles, blocks)
template <int TMAX, typename Fin>
__global__ __launch_bounds__(kWG) void k_beta_vec(DevTables T, const Fin* __restrict__ F,
                                                  int64_t N, double* __restrict__ betaR,
                                                  double* __restrict__ betaL) {
    __shared__ double2 red[(kBetaWaves - 1) * Vec16<Fin>::V * kBetaRhs];
    beta_item_vec<TMAX, Fin>(T, F, N, (int32_t)blockIdx.y, (int64_t)blockIdx.x, betaR, betaL,
                             red);
}

template <int TMAX, typename Fin>
__global__ __launch_bounds__(kWG) void k_beta(DevTables T, const Fin* __restrict__ F, int64_t N,
                                              double* __restrict__ betaR,
                                              double* __restrict__ betaL) {
    __shared__ double2 red[(kBetaWaves - 1) * kBetaRhs];
    beta_item<TMAX, Fin>(T, F, N, (int32_t)blockIdx.y, (int64_t)blockIdx.x, betaR, betaL, red);
}

__global__ __launch_bounds__(kScanRhs * kScanMaxGroupsSingle) void k_iface(
    DevTables T, int64_t N, int32_t per, int32_t G, const double* __restrict__ betaR,
    const double* __restrict__ betaL, double* __restrict__ xsep) {
    extern __shared__ double scan_smem[];
    iface_item<kScanMaxPer>(T, N, per, G, betaR, betaL, xsep, (int64_t)blockIdx.x, scan_smem,
                            kScanRhsLog2);
}

template <int TMAX, typename Fin, typename Xout, int KIND, bool GEN>
__global__ __launch_bounds__(kWG, (sweep_min_waves<KIND, TMAX>())) void k_sweep_reg(
    DevTables T, const Fin* __restrict__ F, Xout* __restrict__ X, int64_t N,
    const double* __restrict__ xsep, int passes) {
    // the refined sweep keeps its FP32 input column in LDS (one row of 256
    // lanes per block row, conflict-free) so that its VGPRs hold only x and
    // the FP32 elimination values
    __shared__ float s_f[KIND == kSweepRefined ? TMAX * kWG : 1];
    // FP32 input: the blocks in reverse, so the rows the beta pass read last
    // are swept first (see k_sweep_halves)
    const int32_t j = std::is_same<Fin, float>::value ? (int32_t)(gridDim.y - 1 - blockIdx.y)
                                                      : (int32_t)blockIdx.y;
    sweep_item<TMAX, Fin, Xout, KIND, GEN>(T, F, X, N, j, (int64_t)blockIdx.x, xsep, passes, s_f);
}

// Sweep of a block in two halves for the modes with FP64 results (tables
// from half_tables): block j's interior rows i0..i1 are a left half of
// kHalfRows rows, the middle row m = i0 + kHalfRows and a right half
// m+1..i1.  Wavefronts 0-1 take the left half of 128 right-hand sides,
// wavefronts 2-3 the right half of the same ones (RHS = 128; with RHS =
// 256, 8 wavefronts of which 0-3 take the left half).
//
// FP64 arithmetic (kSweep64): a twisted factorization of the block, the
// left half eliminated top-down and the right half bottom-up, each with its
// outer boundary value moved into the eliminated right-hand side; row m's
// equation then gives
//     x_m = (f_m - A[m][m-1] dA_{m-1} - A[m][m+1] dB_{m+1}) mid_inv,
// and each half back-substitutes outward from m.  This is a backward-stable
// elimination of the block with known boundary values, like the
// whole-block sweep: its rounding errors stay correlated along the block,
// and the residual stays at the whole-block sweep's level.
//
// Refined (kSweepRefined): each half is solved with zero boundary values
// (refined_solve) and the boundary values enter by superposition:
//     x_m = (f_m - A[m][m-1] qA - A[m][m+1] qB) mid_inv,
//     qA = x0_{m-1} + x(s_j) u_{m-1},  qB = x0_{m+1} + x(s_{j+1}) v_{m+1};
// after the zero-boundary passes one more pass runs on each half with its
// boundary values (refined_boundary_pass, when passes >= 1), so that the
// rounding of the superposition does not stay in the residual.
//
// Each half contributes its term to x_m through LDS and both evaluate the
// same expression (bitwise the same x_m).  Each lane keeps half the rows of
// the whole-block sweep: 4 wavefronts per SIMD instead of 2, which overlap
// their loads, passes and stores.
constexpr int kHalfRhs = 128;        // right-hand sides per workgroup (single matrix)

// one work item of the halves sweep: block j of H's method partition (H.P / 2
// blocks) x RHS right-hand sides from tile * RHS, on 2 RHS threads.  KIND:
// kSweepRefined (FP32 input, refined_solve; s_f: kHalfRows x 2 RHS floats of
// LDS) or kSweep64 (FP64 arithmetic on FP32 or FP64 input, no refinement;
// s_f unused).  s_q: 2 RHS doubles of LDS (refined: 4 RHS, the second
// half for the last pass's exchange).
// The item's two interface values are read before its loads of F, or, with
// a Wait functor whose kFused is true (the fused order), only after the
// zero-boundary solves and a call of wait(), which returns once the
// interface step of these right-hand sides has finished; they are then read
// from the coherence point.
struct NoWait {
    static constexpr bool kFused = false;
    __device__ bool ready() const { return true; }
    __device__ void operator()() const {}
};

template <int RHS, typename Fin, int KIND, bool GEN, typename Wait = NoWait>
__device__ __forceinline__ void halves_item(const DevTables& H, const Fin* __restrict__ F,
                                            double* __restrict__ X, int64_t N, int32_t j,
                                            int64_t tile, const double* __restrict__ xsep,
                                            int passes, float* s_f, double* s_q,
                                            Wait wait = Wait()) {
    double* s_q2 = s_q + 2 * RHS;    // refined: the second exchange
    constexpr int TM = kHalfRows, NT = 2 * RHS;
    const int32_t P = H.P >> 1;                 // blocks of the method's partition
    const int h = __builtin_amdgcn_readfirstlane(threadIdx.x / RHS);   // 0 left, 1 right
    const int c = threadIdx.x % RHS;
    const int64_t n0 = tile * RHS;
    const bool live = n0 + c < N;
    // lanes past N stay for the barrier and re-read the tile's last column
    const int lane = live ? c : (int)(N - 1 - n0);
    const int32_t js = 2 * j + h;
    const int64_t seg_lo = cst(H.starts)[js], seg_hi = cst(H.starts)[js + 1];
    const int64_t i0 = (js == 0) ? seg_lo : seg_lo + 1;
    const int cnt = (int)(seg_hi - i0);         // TM on the left, 1..TM on the right
    // the block's outer boundary value on this half's side
    double xo = 0.0;
    bool early = true;
    if constexpr (Wait::kFused) {
        // the interface values are usually published long before: then they
        // are read here, beside the loads of F, as in the three-launch order
        early = wait.ready();
        if (early) {
            if (h == 0 && j > 0) xo = ld_w<true>(&xsep[(int64_t)(j - 1) * N + n0 + lane]);
            if (h == 1 && j < P - 1) xo = ld_w<true>(&xsep[(int64_t)j * N + n0 + lane]);
        }
    } else {
        if (h == 0 && j > 0) xo = xsep[(int64_t)(j - 1) * N + n0 + lane];
        if (h == 1 && j < P - 1) xo = xsep[(int64_t)j * N + n0 + lane];
    }
    // FP64: slot k of the twisted elimination (tw_* tables) is row i0 + k
    // on the left and row i0 + TM - 1 - k on the right, whose padding slots
    // (k < TM - cnt) re-read its last row
    const int64_t sb = ((int64_t)2 * j + h) * TM;
    Fin f[TM];
    if constexpr (KIND == kSweepRefined) {
        sweep_load<TM, Fin>(F + i0 * N + n0, lane, N, cnt, f);
    } else {
#pragma unroll
        for (int k = 0; k < TM; ++k) {
            const int o = h ? (TM - 1 - k < cnt ? TM - 1 - k : cnt - 1) : k;
            f[k] = (F + (i0 + o) * N + n0)[lane];
        }
    }
    double fm = 0.0;
    if (h == 0) fm = (double)(F + seg_hi * N + n0)[lane];     // row m
    double x[TM];
    if constexpr (KIND == kSweepRefined) {
        float* my_f = s_f + threadIdx.x;
#pragma unroll
        for (int r = 0; r < TM; ++r) my_f[r * NT] = f[r];
        refined_solve<TM, GEN, NT>(H, i0, my_f, passes, x);
    } else {
        // FP64: the twisted elimination toward the middle row, in slot
        // order (x holds the eliminated right-hand side d); a padding slot's
        // successor has coupling zero, so padding never reaches a real row
        const cptr<double> ts = cst(H.tw_s + sb), tr = cst(H.tw_r + sb);
#pragma unroll
        for (int k = 0; k < TM; ++k) {
            const double prev = (k > 0) ? x[k - 1] : 0.0;
            const double sub = (k > 0) ? ts[k] : 0.0;
            x[k] = ((double)f[k] - sub * prev) * tr[k];
        }
    }
    if constexpr (Wait::kFused) {
        if (!__syncthreads_and(early)) {         // one decision for the workgroup
            wait();
            if (h == 0 && j > 0) xo = ld_w<true>(&xsep[(int64_t)(j - 1) * N + n0 + lane]);
            if (h == 1 && j < P - 1) xo = ld_w<true>(&xsep[(int64_t)j * N + n0 + lane]);
        }
    }
    const cptr<double> uu = cst(H.u + i0), vv = cst(H.v + i0);
    if constexpr (KIND == kSweepRefined) {
        // each half's end value next to m in terms of its outer boundary
        if (h == 0)
            s_q[c] = fm - cst(GEN ? H.l64 : H.a64)[seg_hi - 1] * fma(xo, uu[TM - 1], x[TM - 1]);
        else
            s_q[RHS + c] = fma(xo, vv[0], x[0]);
    } else {
        // the outer boundary value enters the eliminated right-hand side
        const cptr<double> te = cst(H.tw_e + sb);
#pragma unroll
        for (int k = 0; k < TM; ++k) x[k] = fma(xo, te[k], x[k]);
        if (h == 0)
            s_q[c] = fm - cst(GEN ? H.l64 : H.a64)[seg_hi - 1] * x[TM - 1];
        else
            s_q[RHS + c] = x[TM - 1];
    }
    __syncthreads();
    const int64_t m = cst(H.starts)[2 * j + 1];
    double xm = (s_q[c] - cst(H.a64)[m] * s_q[RHS + c]) * cst(H.mid_inv)[2 * j + 1];
    double* xb = X + i0 * N + n0;
    if constexpr (KIND == kSweepRefined) {
        // superposition, then (one or more passes) the last pass over the
        // block with its boundary values: each half's residual with x(s_j),
        // x_m or x_m, x(s_{j+1}) eliminated in FP32; row m's correction
        //     dm = (r_m - A[m][m-1] dA_{m-1} - A[m][m+1] dB_{m+1}) mid_inv
        // from the halves' FP32 corrections next to m (one LDS exchange);
        // then each half's back substitution with dm at m, carrying each
        // row's rounded update (carried_back_sub)
        const double xl = h ? xm : xo, xr = h ? xo : xm;
#pragma unroll
        for (int r = 0; r < TM; ++r) x[r] = fma(xr, vv[r], fma(xl, uu[r], x[r]));
        if (passes >= 1) {
            const double a_l = cst(GEN ? H.l64 : H.a64)[m - 1];    // A[m][m-1]
            const double a_r = cst(H.a64)[m];                       // A[m][m+1]
            const double cl = (h == 0 && j == 0) ? 0.0 : cst(GEN ? H.l64 : H.a64)[i0 - 1];
            const double cr = cst(H.a64)[seg_hi - 1];      // zero past the last row
            float w[TM];
            boundary_elim<TM, GEN, NT>(H, i0, s_f + threadIdx.x, cnt, cl, xl, cr, xr, x, w);
            // tables read again here through an offset the compiler cannot
            // see through: kept from the first sweeps, their values would
            // hold some 64 scalar registers across the kernel (spilled)
            asm volatile("" ::: "memory");
            int z;
            asm volatile("s_mov_b32 %0, 0" : "=s"(z));
            const cptr<float> cp32 = cst(H.cp32 + i0) + z, rd32 = cst(H.rd32 + i0) + z;
            if (h == 0) {
                // the left half's last eliminated value is its correction
                // there (its last elimination factor is zero)
                s_q2[c] = fm - a_l * x[TM - 1] - cst(H.b64)[m] * xm - a_l * (double)w[TM - 1];
            } else {
                float d = 0.0f;
#pragma unroll
                for (int r = TM - 1; r >= 0; --r) d = w[r] - cp32[r] * d;
                s_q2[RHS + c] = x[0] + (double)d;
            }
            __syncthreads();
            const double dm = (s_q2[c] - a_r * s_q2[RHS + c]) * cst(H.mid_inv)[2 * j + 1];
            if (h == 1) {
                // dm enters the right half's first row: the eliminated
                // response to it (table eR32; rows past the half's last row
                // read entries of other rows, but never feed a real row)
                const cptr<float> eR = cst(H.eR32 + i0) + z;
                const float dmf = (float)dm;
#pragma unroll
                for (int r = 0; r < TM; ++r) w[r] = fmaf(dmf, eR[r], w[r]);
            }
            carried_back_sub<TM>(H, i0, w, h == 0 ? dm : 0.0,
                                 h == 0 ? cst(H.a64)[m - 1] * (double)rd32[TM - 1] : 0.0, x);
            xm += dm;
        }
        if (!live) return;
#pragma unroll
        for (int r = 0; r < TM; ++r)
            if (r < cnt) store_x(&(xb + (int64_t)r * N)[c], x[r]);
    } else {
        if (!live) return;
        // back substitution outward from m, slots TM-1 .. 0
        const cptr<double> tc = cst(H.tw_c + sb);
        double y = xm;
#pragma unroll
        for (int k = TM - 1; k >= 0; --k) {
            y = fma(-tc[k], y, x[k]);
            const int o = h ? TM - 1 - k : k;
            if (o < cnt) store_x(&(xb + (int64_t)o * N)[c], y);
        }
    }
    if (h == 0) {
        store_x(&X[m * N + n0 + c], xm);
        if (j > 0) store_x(&X[seg_lo * N + n0 + c], xo);
    }
}

template <int RHS, typename Fin, int KIND, bool GEN>
__global__ __launch_bounds__(2 * RHS, 4) void k_sweep_halves(DevTables H,
                                                             const Fin* __restrict__ F,
                                                             double* __restrict__ X, int64_t N,
                                                             const double* __restrict__ xsep,
                                                             int passes) {
    __shared__ float s_f[KIND == kSweepRefined ? kHalfRows * 2 * RHS : 1];
    __shared__ double s_q[(KIND == kSweepRefined ? 4 : 2) * RHS];
    // Order of the work: the blocks in reverse, so the rows the beta pass
    // read last are swept first; k_beta_vec's tiles are this kernel's 128
    // RHS, so tile b runs on the XCD (b % 8) that read its columns in the
    // beta pass.  Poisson 4096 x 4096 on FP32 input: sweep 35.3-36.7 us in
    // the plain order, 33.8 us reversed, 32.1-33.0 us reversed and on the
    // beta pass's XCDs; the bytes fetched past L2 stay the same, so the gain
    // is in how fast those fetches are served.
    const int32_t j = (int32_t)(gridDim.y - 1 - blockIdx.y);
    halves_item<RHS, Fin, KIND, GEN>(H, F, X, N, j, (int64_t)blockIdx.x, xsep, passes, s_f,
                                     s_q);
}

template <typename Fin, typename Xout, int KIND, bool GEN>
__global__ __launch_bounds__(kWG) void k_sweep_stream(DevTables T, const Fin* __restrict__ F,
                                                      Xout* __restrict__ X, int64_t N,
                                                      const double* __restrict__ xsep) {
    sweep_stream_item<Fin, Xout, KIND, GEN>(T, F, X, N, (int32_t)blockIdx.y, (int64_t)blockIdx.x,
                                       xsep);
}

// ==========================================================================
// Fused solve of one matrix whose blocks the sweeps take in halves: the beta
// weights, the interface step and the block sweeps in one launch, with no
// kernel boundary between them.  The series is cut into tiles of kFuseCols
// right-hand sides; tile tau has
//   nb beta items (P blocks x the beta tiles of 64 V columns it holds),
//   ni interface items (dense: column tiles of kDenseCols x row tiles;
//      recurrence: groups of 2^lgR columns, the groups of k_iface),
//   ns = 2 P sweep items (P blocks x two tiles of kHalfRhs columns).
// Every workgroup takes a ticket (one atomic increment) and runs the item the
// ticket names.  Stage s holds, in this order, the interface items of tile
// s - LI, the sweep items of tile s - LS and the beta items of tile s
// (LS = 2 LI, LI = the lag): the beta pass of a tile runs LS stages ahead of its sweeps,
// so the sweeps find its F rows still in a cache and its interface values
// long computed, and reads of F for the weights overlap writes of X.
//
// An interface item waits until the nb beta items of its tile have
// published their weights; a sweep item first solves its halves with zero
// boundary values (the work that does not need the interface values) and
// only then waits until the ni interface items of its tile have published
// theirs.  The items are numbered in that order and a workgroup's ticket
// names two consecutive ones, which it runs in turn.  Every wait is on an
// earlier item: one of a smaller ticket, whose workgroup has started
// (running workgroups take tickets in increasing order), or the same
// workgroup's first item, already done; so the earliest unfinished item can
// always progress and the launch cannot deadlock, however many workgroups
// are resident.  Each wait is bounded all the same (kSpinLimit polls; past it
// the error word is set and the item goes on).  Publishing: the values are
// written through to the device's coherence point (st_w<true>), every wave
// waits for its stores to complete, then one thread increments the tile's
// counter; consumers poll the counter and read with ld_w<true>.  The items
// and their arithmetic are those of k_beta_vec, k_iface / k_iface_dense and
// k_sweep_halves, so X is bitwise that of the three-launch order.
constexpr int64_t kFuseCols = 256;
constexpr int kSpinLimit = 1 << 22;
// every counter of the fused order sits on a line of its own, so that the
// ticket increments, the tile counters' increments and the polls of waiting
// workgroups do not contend for one cache line
constexpr int kSyncStride = 64;   // ints (256 bytes)
// work items per ticket of k_fused and k_fused_batch (their bodies take two)
constexpr int32_t kFusedGroup = 2;

struct FuseShape {
    int64_t T;           // tiles of W right-hand sides
    int32_t W;           // right-hand sides per tile (a multiple of kFuseCols)
    int32_t LI, LS;      // stage lags of the interface and sweep items
    int32_t nb, ni, ns;  // items per tile
    int32_t rowtiles;    // dense row tiles (1: recurrence order)
    int32_t bpt;         // beta tiles per fuse tile
    int32_t spt;         // sweep tiles (kHalfRhs columns) per fuse tile
};

__device__ __forceinline__ int64_t fuse_stage_size(const FuseShape& f, int64_t s) {
    int64_t z = 0;
    if (s >= f.LI && s - f.LI < f.T) z += f.ni;
    if (s >= f.LS && s - f.LS < f.T) z += f.ns;
    if (s < f.T) z += f.nb;
    return z;
}

// wait until *cnt >= target (thread 0 polls; the workgroup then proceeds)
__device__ __forceinline__ void fuse_wait(const int* cnt, int target, int* err) {
    if (threadIdx.x == 0) {
        int polls = 0;
        while (__hip_atomic_load(const_cast<int*>(cnt), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++polls > kSpinLimit) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
    }
    __syncthreads();
}

// publish: every wave's stores have completed, then one increment
__device__ __forceinline__ void fuse_signal(int* cnt) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct FuseWait {
    static constexpr bool kFused = true;
    const int* cnt;
    int target;
    int* err;
    // one look at the counter, no wait (every lane loads the same word)
    __device__ bool ready() const {
        return __hip_atomic_load(const_cast<int*>(cnt), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) >= target;
    }
    __device__ void operator()() const { fuse_wait(cnt, target, err); }
};

// LDS of a fused workgroup (doubles): the largest of the halves sweep
// (refined: kHalfRows x 2 kHalfRhs floats of F, then 4 kHalfRhs doubles;
// FP64 arithmetic: 2 kHalfRhs doubles), the beta reduction and the
// 256-thread interface scan
constexpr int kFuseSweepLds = kHalfRows * kHalfRhs + 4 * kHalfRhs;
constexpr int kFuseSweep64Lds = 2 * kHalfRhs;
constexpr int kFuseScanLds = 2 * kScanBatchThreads + 2 * kScanMaxGroupsSingle +
                             kScanBatchThreads * kScanMaxPer;
constexpr int kFuseBetaLds = 2 * (kBetaWaves - 1) * 4 * kBetaRhs;
constexpr int kFuseDenseBatch = 16;   // k-steps per operand load (register budget)

// sync: lines (kSyncStride ints) of [0] the ticket, [1] the error word,
// [2, 2 + T) the beta counters, [2 + T, 2 + 2T) the interface counters;
// zero before the launch.
// One work item of k_fused: item `rem` in ticket order.
template <typename Fin, int KIND, bool DENSE, bool GEN>
__device__ __forceinline__ void fused_item(
    const DevTables& T, const DevTables& H, const Fin* __restrict__ F, double* __restrict__ X,
    int64_t N, double* betaR, double* betaL, double* xsep, const double* __restrict__ Kt,
    int32_t Pc, int32_t Mr, int32_t per, int32_t G, int32_t lgR, int passes,
    const FuseShape& fs, int* sync, int64_t rem, double* smem) {
    int* err = sync + kSyncStride;
    int* beta_done = sync + 2 * kSyncStride;                  // line 2 + tau
    int* iface_done = sync + (2 + fs.T) * kSyncStride;        // line 2 + T + tau
    // ticket -> (stage, index in stage): stage sizes are constant between
    // the breakpoints 0, LI, LS, T, T + LI, T + LS
    int64_t bp[6] = {0, fs.LI, fs.LS, fs.T, fs.T + fs.LI, fs.T + fs.LS};
    for (int a = 1; a < 6; ++a)
        for (int b = a; b > 0 && bp[b - 1] > bp[b]; --b) {
            const int64_t tmp = bp[b];
            bp[b] = bp[b - 1];
            bp[b - 1] = tmp;
        }
    int64_t stage = -1, idx = 0;
    for (int k = 0; k < 5 && stage < 0; ++k) {
        const int64_t lo = bp[k], hi = bp[k + 1];
        if (hi <= lo) continue;
        const int64_t sz = fuse_stage_size(fs, lo);
        if (sz == 0) continue;
        if (rem < (hi - lo) * sz) {
            stage = lo + rem / sz;
            idx = rem % sz;
        } else {
            rem -= (hi - lo) * sz;
        }
    }
    if (stage < 0) return;                       // past the last item (not launched)
    const int32_t P = T.P;
    // interface items of tile stage - LI
    if (stage >= fs.LI && stage - fs.LI < fs.T) {
        if (idx < fs.ni) {
            const int64_t tau = stage - fs.LI;
            fuse_wait(beta_done + tau * kSyncStride, fs.nb, err);
            if constexpr (DENSE) {
                const int64_t ct = tau * (fs.W / kDenseCols) + idx / fs.rowtiles;
                dense_item<kFuseDenseBatch, true>(Kt, Pc, Mr, P, N, betaR, betaL, xsep, ct,
                                                  (int32_t)(idx % fs.rowtiles));
            } else {
                const int64_t sblk = ((tau * fs.W) >> lgR) + idx;
                iface_item<kScanMaxPer, true>(T, N, per, G, betaR, betaL, xsep, sblk, smem, lgR);
            }
            fuse_signal(iface_done + tau * kSyncStride);
            return;
        }
        idx -= fs.ni;
    }
    // sweep items of tile stage - LS: block-major, neighbouring column
    // tiles of one block next to each other (consecutive workgroups read
    // and write adjacent spans of the same rows)
    if (stage >= fs.LS && stage - fs.LS < fs.T) {
        if (idx < fs.ns) {
            const int64_t tau = stage - fs.LS;
            const int64_t ht = tau * fs.spt + idx % fs.spt;     // tile of kHalfRhs columns
            if (ht * kHalfRhs >= N) return;
            FuseWait w{iface_done + tau * kSyncStride, fs.ni, err};
            halves_item<kHalfRhs, Fin, KIND, GEN, FuseWait>(
                H, F, X, N, (int32_t)(idx / fs.spt), ht, xsep, passes, (float*)smem,
                KIND == kSweepRefined ? smem + kHalfRows * kHalfRhs : smem, w);
            return;
        }
        idx -= fs.ns;
    }
    // beta items of tile stage, block-major as the sweeps
    {
        const int64_t tau = stage;
        const int64_t bt = tau * fs.bpt + idx % fs.bpt;
        beta_item_vec<64, Fin, true>(T, F, N, (int32_t)(idx / fs.bpt), bt, betaR, betaL,
                                     (double2*)smem);
        fuse_signal(beta_done + tau * kSyncStride);
    }
}

// Workgroups increment the one ticket counter, and those increments are
// serialised (some 12-14 ns each): a ticket takes kFusedGroup = 2
// consecutive items, in order (a wait of the second is on earlier tickets
// or on the first, already done).
template <typename Fin, int KIND, bool DENSE, bool GEN>
__global__ __launch_bounds__(2 * kHalfRhs, 4) void k_fused(
    DevTables T, DevTables H, const Fin* __restrict__ F, double* __restrict__ X, int64_t N,
    double* betaR, double* betaL, double* xsep, const double* __restrict__ Kt, int32_t Pc,
    int32_t Mr, int32_t per, int32_t G, int32_t lgR, int passes, FuseShape fs, int* sync,
    int64_t items) {
    static_assert(2 * kHalfRhs == kWG, "one workgroup shape for every item");
    constexpr int LS = KIND == kSweepRefined ? kFuseSweepLds : kFuseSweep64Lds;
    constexpr int L0 = LS > kFuseBetaLds ? LS : kFuseBetaLds;
    constexpr int LDS = DENSE ? L0 : (L0 > kFuseScanLds ? L0 : kFuseScanLds);
    __shared__ double smem[LDS];
    __shared__ int64_t s_ticket;
    if (threadIdx.x == 0)
        s_ticket = __hip_atomic_fetch_add(sync, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int64_t q0 = s_ticket * kFusedGroup;
    fused_item<Fin, KIND, DENSE, GEN>(T, H, F, X, N, betaR, betaL, xsep, Kt, Pc, Mr, per, G, lgR,
                                      passes, fs, sync, q0, smem);
    if (q0 + 1 < items) {
        __syncthreads();                        // LDS of the first item
        fused_item<Fin, KIND, DENSE, GEN>(T, H, F, X, N, betaR, betaL, xsep, Kt, Pc, Mr, per, G,
                                          lgR, passes, fs, sync, q0 + 1, smem);
    }
}

__global__ void k_zero_i32(int* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ==========================================================================
// batch kernels: one 1-D launch per step over the work items of all
// matrices; item ranges per matrix are prefix sums in the descriptors, and
// own[item] names the matrix of each item (one scalar load in place of a
// binary search over the descriptors, whose chain of dependent loads held
// every workgroup for microseconds before its first load of F).

// Item of a batch workgroup.  Workgroups are dispatched to the chip's 8
// XCDs (each with its own L2) round-robin by index; consecutive items are
// neighbouring tiles of one block, whose rows share cache lines at the tile
// boundaries when N is not a multiple of 32 (F) or 16 (X).  Runs of
// kXcdRun consecutive items go to one XCD, and the XCDs take the runs in
// turn: most neighbours then share an L2, so such a line is fetched once,
// while every XCD still works through the whole batch at the same pace (one
// contiguous share per XCD removed the extra fetches but lost more to the
// uneven cost of the shares).  A bijection of [0, gridDim.x): the last,
// partial group of 8 runs keeps the plain order.
constexpr uint32_t kXcds = 8;
constexpr uint32_t kXcdRun = 8;
__device__ __forceinline__ int64_t xcd_item() {
    const uint32_t n = gridDim.x, x = blockIdx.x;
    constexpr uint32_t span = kXcds * kXcdRun;
    const uint32_t sup = x / span, within = x % span;
    if ((uint64_t)(sup + 1) * span > n) return x;
    return (int64_t)sup * span + (within % kXcds) * kXcdRun + within / kXcds;
}

// one workgroup per item: wavefront wv takes right-hand sides wv*64 .. +63
// of the item's 256 (beta_rows_item)
template <int TMAX, typename Fin>
__global__ __launch_bounds__(kWG) void k_beta_batch(const BatchDesc* __restrict__ D,
                                                    const int32_t* __restrict__ own) {
    const int64_t item = xcd_item();
    const int32_t k = cst(own)[item];
    const BatchDesc d = D[k];    // uniform, before any store: scalar loads
    const int64_t local = item - d.item0;
    const int64_t tiles = (d.N + kWG - 1) / kWG;
    if (d.T.P < 2 || local >= (int64_t)d.T.P * tiles) return;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kBetaRhs);
    beta_rows_item<TMAX, Fin>(d.T, (const Fin*)d.F, d.N, (int32_t)(local / tiles),
                              (local % tiles) * kWG + wv * kBetaRhs, d.betaR, d.betaL);
}

// one workgroup of kScanBatchWide per R_k right-hand sides of matrix k
// (G_k R_k <= kScanBatchWide); LDS for the largest shape, G R =
// kScanBatchWide with per <= kScanMaxPer
__global__ __launch_bounds__(kScanBatchWide) void k_iface_batch(
    const BatchDesc* __restrict__ D, const int32_t* __restrict__ own) {
    // carries 2 G R + factors 2 G + S^R by row G per R, with G R <= 256
    __shared__ double S[2 * kScanBatchWide + 2 * kScanMaxGroupsSingle +
                        kScanBatchWide * kScanMaxPer];
    const int64_t item = xcd_item();
    const int32_t k = cst(own)[item];
    const BatchDesc d = D[k];    // uniform, before any store: scalar loads
    const int64_t local = item - d.scan0;
    if (d.T.P < 2 || (local << d.lgR) >= d.N) return;   // uniform per workgroup
    iface_item<kScanMaxPer>(d.T, d.N, d.per, d.G, d.betaR, d.betaL, d.xsep, local, S, d.lgR);
}

template <int TMAX, typename Fin, typename Xout, int KIND>
__global__ __launch_bounds__(kWG, (sweep_min_waves<KIND, TMAX>())) void k_sweep_batch(
    const BatchDesc* __restrict__ D, const int32_t* __restrict__ own, int passes) {
    __shared__ float s_f[KIND == kSweepRefined ? TMAX * kWG : 1];
    const int64_t item = xcd_item();
    const int32_t k = cst(own)[item];
    const BatchDesc d = D[k];    // uniform, before any store: scalar loads
    const int64_t local = item - d.item0;
    const int64_t tiles = (d.N + kWG - 1) / kWG;
    if (local >= (int64_t)d.T.P * tiles) return;
    sweep_item<TMAX, Fin, Xout, KIND, false>(d.T, (const Fin*)d.F, (Xout*)d.X, d.N,
                                      (int32_t)(local / tiles), local % tiles, d.xsep, passes,
                                      s_f);
}

// the batch's refined or FP64-arithmetic sweep when every matrix takes its
// blocks in halves (BatchDesc::H): one workgroup of 2 x 256 threads per item,
// the item structure of k_sweep_batch
template <typename Fin, int KIND>
__global__ __launch_bounds__(2 * kWG, 4) void k_sweep_batch_halves(const BatchDesc* __restrict__ D,
                                                                   const int32_t* __restrict__ own,
                                                                   int passes) {
    __shared__ float s_f[KIND == kSweepRefined ? kHalfRows * 2 * kWG : 1];
    __shared__ double s_q[(KIND == kSweepRefined ? 4 : 2) * kWG];
    const int64_t item = xcd_item();
    const int32_t k = cst(own)[item];
    const BatchDesc d = D[k];    // uniform, before any store: scalar loads
    const int64_t local = item - d.item0;
    const int64_t tiles = (d.N + kWG - 1) / kWG;
    if (local >= (int64_t)d.T.P * tiles) return;        // uniform per workgroup
    halves_item<kWG, Fin, KIND, false>(d.H, (const Fin*)d.F, (double*)d.X, d.N,
                                       (int32_t)(local / tiles), local % tiles, d.xsep, passes,
                                       s_f, s_q);
}

// The uneven batch in one launch (tdsolve_batch_set_fused): the beta,
// interface and sweep items of every matrix in one grid, taken in ticket
// order, two consecutive items per ticket.  Stages are the tiles of kWG
// columns of every matrix, matrix by matrix: stage s holds the interface
// items of tile s - LI, the sweep items of tile s - LS and the beta items of
// tile s (LS = 2 LI), and the host writes the items in that order into tk
// (the kind in bits 62-63, the matrix in bits 32-61, the item's index
// within its matrix in bits 0-31).
// An interface item waits until the P beta items of its tile have published
// their weights, a sweep item until the interface items of its tile have
// published their values; every wait is on items earlier in tk, held by
// smaller tickets or done by the same workgroup before, so the launch
// cannot deadlock (the argument of k_fused), and every wait is bounded.
// The items are those of k_beta_batch, k_iface_batch (on 256 threads: half
// its right-hand sides per workgroup, the same groups of blocks, so bitwise
// the same values; 2^lgR divides kWG, so an item never spans two tiles) and
// k_sweep_batch, so X is bitwise that of the separate launches.  Matrices
// whose blocks fit 32 rows.  sync: lines of kSyncStride ints: [0] the
// ticket, [1] the error word, [2, 2 + S) the beta counters of the S tiles,
// [2 + S, 2 + 2S) their interface counters; zero before the launch.
// one work item of k_fused_batch (code: its entry of the ticket table)
template <typename Fin, typename Xout, int KIND>
__device__ __forceinline__ void fused_batch_item(const BatchDesc* __restrict__ D, uint64_t code,
                                                 int64_t S, int passes, int* __restrict__ sync,
                                                 double* smem) {
    const uint64_t kind = code >> 62;
    const int32_t k = (int32_t)((code >> 32) & 0x3fffffffu);
    const int64_t local = (int64_t)(code & 0xffffffffu);
    const BatchDesc d = D[k];    // uniform, before any store: scalar loads
    int* err = sync + kSyncStride;
    int* beta_done = sync + 2 * kSyncStride;            // + tile * kSyncStride
    int* iface_done = sync + (2 + S) * kSyncStride;
    const int64_t tiles = (d.N + kWG - 1) / kWG;
    const int lgR = d.lgR - 1;                  // G R <= 256 (k_iface_batch: <= 512)
    if (kind == kFusedBeta) {
        const int64_t tau = local % tiles;
        const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kBetaRhs);
        beta_rows_item<32, Fin, true>(d.T, (const Fin*)d.F, d.N, (int32_t)(local / tiles),
                                      tau * kWG + wv * kBetaRhs, d.betaR, d.betaL);
        fuse_signal(beta_done + (d.tile0 + tau) * kSyncStride);
    } else if (kind == kFusedIface) {
        const int64_t tau = (local << lgR) / kWG;
        fuse_wait(beta_done + (d.tile0 + tau) * kSyncStride, d.T.P, err);
        iface_item<kScanMaxPer, true>(d.T, d.N, d.per, d.G, d.betaR, d.betaL, d.xsep, local,
                                      smem, lgR);
        fuse_signal(iface_done + (d.tile0 + tau) * kSyncStride);
    } else {
        const int64_t tau = local % tiles;
        if (d.T.P > 1) {
            // the interface items of columns tau kWG .. min((tau + 1) kWG, N) - 1
            const int64_t c1 = min((tau + 1) * kWG, d.N);
            const int64_t want = ((c1 + ((int64_t)1 << lgR) - 1) >> lgR) - ((tau * kWG) >> lgR);
            fuse_wait(iface_done + (d.tile0 + tau) * kSyncStride, (int)want, err);
        }
        sweep_item<32, Fin, Xout, KIND, false, true>(d.T, (const Fin*)d.F, (Xout*)d.X, d.N,
                                                     (int32_t)(local / tiles), tau, d.xsep,
                                                     passes, (float*)smem);
    }
}

template <typename Fin, typename Xout, int KIND>
__global__ __launch_bounds__(kWG, (sweep_min_waves<KIND, 32>())) void k_fused_batch(
    const BatchDesc* __restrict__ D, const uint64_t* __restrict__ tk, int64_t nitems,
    int64_t S, int passes, int* __restrict__ sync) {
    // LDS: the refined sweep's F (32 rows x 256 floats) or the interface scan
    constexpr int LSW = KIND == kSweepRefined ? 32 * kWG / 2 : 1;
    __shared__ double smem[LSW > kFuseScanLds ? LSW : kFuseScanLds];
    __shared__ int32_t s_ticket;
    if (threadIdx.x == 0)
        s_ticket = __hip_atomic_fetch_add(sync, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    // one ticket: kFusedGroup consecutive items of the table, in order (a
    // wait of the later one is on earlier tickets or on this workgroup's own
    // finished item).  Every workgroup increments the one ticket counter,
    // which serialises them: one item per ticket, the refined batch took
    // 3.68 ms per step at best, two 3.26 ms; three or four hold more
    // registers across the items and spill (3.66 and 3.71 ms).
    const int64_t q0 = (int64_t)__builtin_amdgcn_readfirstlane(s_ticket) * kFusedGroup;
    fused_batch_item<Fin, Xout, KIND>(D, cst(tk)[q0], S, passes, sync, smem);
    if (q0 + 1 < nitems) {
        __syncthreads();                        // LDS of the first item
        fused_batch_item<Fin, Xout, KIND>(D, cst(tk)[q0 + 1], S, passes, sync, smem);
    }
}

// ==========================================================================
// launchers

// a kernel launch; with `tm`, its start and stop events take the kernel's
// own start and end timestamps (phase timing without the dispatch gaps)
template <typename Kern, typename... Args>
static void launch_k(Kern kernel, dim3 g, dim3 b, uint32_t lds, hipStream_t s, const KTime* tm,
                     Args... args) {
    if (tm)
        hipExtLaunchKernelGGL(kernel, g, b, lds, s, tm->start, tm->stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, g, b, lds, s, args...);
}
static inline dim3 grid2(int64_t N, int64_t y) {
    return dim3((unsigned)((N + kWG - 1) / kWG), (unsigned)y, 1);
}

int32_t rows_bucket(int32_t max_rows) {
    return max_rows <= 32 ? 32 : max_rows <= 64 ? 64 : max_rows <= 128 ? 128 : 0;
}

hipError_t launch_beta(const DevTables& t, const void* F, bool f32, int64_t N, double* betaR,
                       double* betaL, hipStream_t s, const KTime* tm) {
    if (t.P < 2 || N == 0) return hipSuccess;
    // two right-hand sides per lane, loads of 8 (FP32) or 16 (FP64) bytes
    const int V = 2;
    const uintptr_t align = f32 ? 7 : 15;
    if (N % V == 0 && ((uintptr_t)F & align) == 0 &&
        (t.wpad_rows == 32 || t.wpad_rows == 64 || t.wpad_rows == 128)) {
        const dim3 gv((unsigned)((N + V * kBetaRhs - 1) / (V * kBetaRhs)), (unsigned)t.P, 1);
#define TDS_BETA_VEC(TM, FT) \
    launch_k(k_beta_vec<TM, FT>, gv, dim3(kWG), 0, s, tm, t, (const FT*)F, N, betaR, betaL)
        if (t.wpad_rows == 32) {
            if (f32) TDS_BETA_VEC(32, float); else TDS_BETA_VEC(32, double);
        } else if (t.wpad_rows == 64) {
            if (f32) TDS_BETA_VEC(64, float); else TDS_BETA_VEC(64, double);
        } else {
            if (f32) TDS_BETA_VEC(128, float); else TDS_BETA_VEC(128, double);
        }
#undef TDS_BETA_VEC
        return hipGetLastError();
    }
    const dim3 g((unsigned)((N + kBetaRhs - 1) / kBetaRhs), (unsigned)t.P, 1);
#define TDS_BETA(TM, FT) \
    launch_k(k_beta<TM, FT>, g, dim3(kWG), 0, s, tm, t, (const FT*)F, N, betaR, betaL)
    switch (t.wpad_rows) {
        case 32:
            if (f32) TDS_BETA(32, float); else TDS_BETA(32, double);
            break;
        case 64:
            if (f32) TDS_BETA(64, float); else TDS_BETA(64, double);
            break;
        case 128:
            if (f32) TDS_BETA(128, float); else TDS_BETA(128, double);
            break;
        default:
            if (f32) TDS_BETA(0, float); else TDS_BETA(0, double);
            break;
    }
#undef TDS_BETA
    return hipGetLastError();
}

void batch_scan_shape(int32_t P, int32_t* per, int32_t* G, int32_t* lgR) {
    // the groups of the single-matrix scan (scan_shape: at least 4 blocks
    // per group, at most kScanMaxGroupsSingle groups), so that a matrix's
    // interface values are bitwise those of its single plan, on a workgroup
    // of kScanBatchWide: G groups x R = 2^lgR right-hand sides, R the
    // largest power of two with G R <= kScanBatchWide.  Small systems get
    // many right-hand sides per workgroup, large ones many short groups.
    scan_shape(P, kScanMaxGroupsSingle, per, G);
    int32_t lg = 0;
    while ((1 << (lg + 1)) * *G <= kScanBatchWide) ++lg;
    *lgR = lg;
}

void scan_shape(int32_t P, int32_t max_groups, int32_t* per, int32_t* G) {
    const int32_t nsep = P > 1 ? P - 1 : 1;
    int32_t p = (nsep + max_groups - 1) / max_groups;
    if (p < 4) p = 4;
    *per = p;
    *G = (nsep + p - 1) / p;
}

hipError_t launch_iface(const DevTables& t, const double* betaR, const double* betaL,
                        double* xsep, int64_t N, hipStream_t s, const KTime* tm) {
    if (t.P < 2 || N == 0) return hipSuccess;
    int32_t per, G;
    scan_shape(t.P, kScanMaxGroupsSingle, &per, &G);
    const size_t lds = sizeof(double) * scan_lds_doubles(G, per);
    launch_k(k_iface, dim3((unsigned)((N + kScanRhs - 1) / kScanRhs)),
                       dim3(kScanRhs * G), lds, s, tm, t, N, per, G, betaR, betaL, xsep);
    return hipGetLastError();
}

hipError_t launch_iface_dense(const double* Kt, int32_t Pc, int32_t Mr, int32_t P,
                              const double* betaR, const double* betaL, double* xsep, int64_t N,
                              hipStream_t s, const KTime* tm) {
    if (P < 2 || N == 0) return hipSuccess;
    if (Pc % 4 != 0 || Pc < P || Mr % kDenseRows != 0 || Mr < P - 1) return hipErrorInvalidValue;
    const dim3 g((unsigned)((N + kDenseCols - 1) / kDenseCols),
                 (unsigned)((P - 1 + kDenseRows - 1) / kDenseRows), 1);
    launch_k(k_iface_dense, g, dim3(kWG), 0, s, tm, Kt, Pc, Mr, P, N, betaR, betaL, xsep);
    return hipGetLastError();
}

hipError_t launch_iface_dichotomy(const DevTables& t, const double* betaR, const double* betaL,
                                  double* SR, double* SL, double* xsep, int64_t N,
                                  hipStream_t s, const KTime* tm) {
    if (t.P < 2 || N == 0) return hipSuccess;
    launch_k(k_iface_dich, dim3((unsigned)((N + kDichRhs - 1) / kDichRhs)), dim3(kWG), 0, s, tm,
             t, N, betaR, betaL, SR, SL, xsep);
    return hipGetLastError();
}

template <typename Fin, typename Xout, int KIND, bool GEN>
static void go_sweep_t(const DevTables& t, const void* F, void* X, int64_t N, int passes,
                       const double* xsep, hipStream_t s, const KTime* tm,
                       const DevTables* halves) {
    const int m = t.max_rows;
    const dim3 g = grid2(N, t.P);
    if constexpr (KIND == kSweepRefined || (KIND == kSweep64 && std::is_same<Xout, double>::value)) {
        if (halves && m > kHalfRows && m <= 2 * kHalfRows && halves->P == 2 * t.P) {
            launch_k(k_sweep_halves<kHalfRhs, Fin, KIND, GEN>,
                     dim3((unsigned)((N + kHalfRhs - 1) / kHalfRhs), t.P, 1), dim3(2 * kHalfRhs),
                     0, s, tm, *halves, (const Fin*)F, (double*)X, N, xsep, passes);
            return;
        }
    }
#define TDS_SWEEP(TM)                                                                   \
    launch_k(k_sweep_reg<TM, Fin, Xout, KIND, GEN>, g, dim3(kWG), 0, s, tm, t, (const Fin*)F, \
             (Xout*)X, N, xsep, passes)
    if (m <= 16)
        TDS_SWEEP(16);
    else if (m <= 32)
        TDS_SWEEP(32);
    else if (m <= 64)
        TDS_SWEEP(64);
    else if (m <= kRegMaxRows && KIND != kSweepRefined)
        TDS_SWEEP(128);
    else if (m <= kRegMaxRows)
        // the refined sweep's registers hold 64-row blocks; longer ones take
        // the register sweep in FP64 arithmetic (as accurate, no passes)
        launch_k(k_sweep_reg<128, Fin, Xout, kSweep64, GEN>, g, dim3(kWG), 0, s, tm, t,
                 (const Fin*)F, (Xout*)X, N, xsep, passes);
    else
        launch_k(k_sweep_stream<Fin, Xout, KIND == kSweep32 ? kSweep32 : kSweep64, GEN>, g,
                 dim3(kWG), 0, s, tm, t, (const Fin*)F, (Xout*)X, N, xsep);
#undef TDS_SWEEP
}

template <typename Fin, typename Xout, int KIND>
static void go_sweep(const DevTables& t, const void* F, void* X, int64_t N, int passes,
                     const double* xsep, hipStream_t s, const KTime* tm,
                     const DevTables* halves) {
    if (t.general)
        go_sweep_t<Fin, Xout, KIND, true>(t, F, X, N, passes, xsep, s, tm, halves);
    else
        go_sweep_t<Fin, Xout, KIND, false>(t, F, X, N, passes, xsep, s, tm, halves);
}

hipError_t launch_sweep(const DevTables& t, const void* F, void* X, int64_t N, int mode,
                        int passes, const double* xsep, hipStream_t s, const KTime* tm,
                        const DevTables* halves) {
    if (N == 0) return hipSuccess;
    switch (mode) {
        case TDS_F64:
            go_sweep<double, double, kSweep64>(t, F, X, N, passes, xsep, s, tm, halves);
            break;
        case TDS_F32_WIDE:
            go_sweep<float, double, kSweep64>(t, F, X, N, passes, xsep, s, tm, halves);
            break;
        case TDS_F32:
            go_sweep<float, float, kSweep32>(t, F, X, N, passes, xsep, s, tm, nullptr);
            break;
        case TDS_F32_REFINED:
            go_sweep<float, double, kSweepRefined>(t, F, X, N, passes, xsep, s, tm, halves);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool fused_fits(const DevTables& t, const DevTables* halves, const void* F, int64_t N, int mode,
                int order) {
    if (mode == TDS_F32 || order == TDS_IFACE_DICHOTOMY || t.P < 2 || N == 0) return false;
    if (!halves || halves->P != 2 * t.P || t.wpad_rows != 64) return false;
    if (t.max_rows <= kHalfRows || t.max_rows > 2 * kHalfRows) return false;
    return N % 2 == 0 && ((uintptr_t)F & (mode == TDS_F64 ? 15 : 7)) == 0;
}

int64_t fused_sync_ints(int64_t N) {
    // tiles of at least kFuseCols columns: room for any tile width
    return kSyncStride * (2 + 2 * ((N + kFuseCols - 1) / kFuseCols));
}

template <typename Fin, int KIND, bool DENSE, bool GEN>
static hipError_t fused_t(const DevTables& t, const DevTables& h, const void* F, void* X,
                          int64_t N, int passes, double* betaR, double* betaL, double* xsep,
                          const double* Kt, int32_t Pc, int32_t Mr, int32_t lag, int32_t W,
                          int* sync, hipStream_t s, const KTime* tm) {
    constexpr int32_t V = Vec16<Fin>::V;       // right-hand sides per lane of a beta item
    FuseShape fs;
    fs.W = W;
    fs.T = (N + W - 1) / W;
    // the interface items of a tile `lag` stages after its beta items, its
    // sweeps `lag` stages later still: long enough that the items waited on
    // have left the resident window (measured: an interface lag of 1 stage
    // made the kernel 1.5x slower than 5-8 stages)
    fs.LI = lag;
    fs.LS = 2 * lag;
    fs.bpt = (int32_t)(W / (V * kBetaRhs));
    fs.spt = (int32_t)(W / kHalfRhs);
    fs.nb = t.P * fs.bpt;
    fs.ns = t.P * fs.spt;
    int32_t per = 0, G = 0, lgR = 0;
    if (DENSE) {
        fs.rowtiles = (t.P - 1 + kDenseRows - 1) / kDenseRows;
        fs.ni = (int32_t)(W / kDenseCols) * fs.rowtiles;
    } else {
        // the groups of k_iface (scan_shape), on 256 threads: G groups x
        // 2^lgR right-hand sides; the same carries, bitwise the same values
        scan_shape(t.P, kScanMaxGroupsSingle, &per, &G);
        while ((1 << (lgR + 1)) * G <= kScanBatchThreads) ++lgR;
        fs.rowtiles = 1;
        fs.ni = (int32_t)(W >> lgR);
    }
    const int64_t items = fs.T * (int64_t)(fs.nb + fs.ni + fs.ns);
    if (items > INT32_MAX) return hipErrorInvalidValue;
    const int64_t nsync = kSyncStride * (2 + 2 * fs.T);
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((nsync + kWG - 1) / kWG)), dim3(kWG), 0, s,
                       sync, nsync);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    launch_k(k_fused<Fin, KIND, DENSE, GEN>,
             dim3((unsigned)((items + kFusedGroup - 1) / kFusedGroup)), dim3(2 * kHalfRhs), 0, s,
             tm, t, h, (const Fin*)F, (double*)X, N, betaR, betaL, xsep, Kt, Pc, Mr, per, G, lgR,
             passes, fs, sync, items);
    return hipGetLastError();
}

template <typename Fin, int KIND, bool DENSE>
static hipError_t fused_g(const DevTables& t, const DevTables& h, const void* F, void* X,
                          int64_t N, int passes, double* betaR, double* betaL, double* xsep,
                          const double* Kt, int32_t Pc, int32_t Mr, int32_t lag, int32_t W,
                          int* sync, hipStream_t s, const KTime* tm) {
    if (t.general)
        return fused_t<Fin, KIND, DENSE, true>(t, h, F, X, N, passes, betaR, betaL, xsep, Kt, Pc,
                                               Mr, lag, W, sync, s, tm);
    return fused_t<Fin, KIND, DENSE, false>(t, h, F, X, N, passes, betaR, betaL, xsep, Kt, Pc,
                                            Mr, lag, W, sync, s, tm);
}

template <bool DENSE>
static hipError_t fused_m(const DevTables& t, const DevTables& h, const void* F, void* X,
                          int64_t N, int mode, int passes, double* betaR, double* betaL,
                          double* xsep, const double* Kt, int32_t Pc, int32_t Mr, int32_t lag,
                          int32_t W, int* sync, hipStream_t s, const KTime* tm) {
    switch (mode) {
        case TDS_F64:
            return fused_g<double, kSweep64, DENSE>(t, h, F, X, N, passes, betaR, betaL, xsep, Kt,
                                                    Pc, Mr, lag, W, sync, s, tm);
        case TDS_F32_WIDE:
            return fused_g<float, kSweep64, DENSE>(t, h, F, X, N, passes, betaR, betaL, xsep, Kt,
                                                   Pc, Mr, lag, W, sync, s, tm);
        case TDS_F32_REFINED:
            return fused_g<float, kSweepRefined, DENSE>(t, h, F, X, N, passes, betaR, betaL,
                                                        xsep, Kt, Pc, Mr, lag, W, sync, s, tm);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fused(const DevTables& t, const DevTables& h, const void* F, void* X,
                        int64_t N, int mode, int passes, double* betaR, double* betaL,
                        double* xsep, const double* Kt, int32_t Pc, int32_t Mr, int32_t lag,
                        int32_t W, int* sync, hipStream_t s, const KTime* tm) {
    if (lag < 1 || !sync || W < kFuseCols || W % kFuseCols != 0) return hipErrorInvalidValue;
    if (Kt && (Pc % 4 != 0 || Pc < t.P || Mr % kDenseRows != 0 || Mr < t.P - 1))
        return hipErrorInvalidValue;
    if (Kt)
        return fused_m<true>(t, h, F, X, N, mode, passes, betaR, betaL, xsep, Kt, Pc, Mr, lag, W,
                             sync, s, tm);
    return fused_m<false>(t, h, F, X, N, mode, passes, betaR, betaL, xsep, Kt, Pc, Mr, lag, W,
                          sync, s, tm);
}

template <int TM>
static void batch_sweep(const BatchDesc* D, const int32_t* own, int64_t items, int mode,
                        int passes, bool halves, hipStream_t s, const KTime* tm) {
    const dim3 g((unsigned)items);
    if (TM == 64 && halves && mode != TDS_F32) {
        if (mode == TDS_F32_REFINED)
            launch_k(k_sweep_batch_halves<float, kSweepRefined>, g, dim3(2 * kWG), 0, s, tm, D, own,
                     passes);
        else if (mode == TDS_F64)
            launch_k(k_sweep_batch_halves<double, kSweep64>, g, dim3(2 * kWG), 0, s, tm, D, own,
                     passes);
        else
            launch_k(k_sweep_batch_halves<float, kSweep64>, g, dim3(2 * kWG), 0, s, tm, D, own,
                     passes);
        return;
    }
    switch (mode) {
        case TDS_F64:
            launch_k(k_sweep_batch<TM, double, double, kSweep64>, g, dim3(kWG), 0, s, tm,
                     D, own, passes);
            break;
        case TDS_F32_WIDE:
            launch_k(k_sweep_batch<TM, float, double, kSweep64>, g, dim3(kWG), 0, s, tm,
                     D, own, passes);
            break;
        case TDS_F32:
            launch_k(k_sweep_batch<TM, float, float, kSweep32>, g, dim3(kWG), 0, s, tm,
                     D, own, passes);
            break;
        default:
            launch_k(k_sweep_batch<TM, float, double, kSweepRefined>, g, dim3(kWG), 0, s, tm, D,
                     own, passes);
            break;
    }
}

hipError_t launch_batch(const BatchDesc* D, const int32_t* own_items, const int32_t* own_scans,
                        int64_t items32, int64_t items64, int64_t scans, int mode, int passes,
                        bool halves, const KTime* tm, hipStream_t s) {
    if (items32 + items64 == 0) return hipSuccess;
    if (items32 > INT32_MAX || items64 > INT32_MAX || scans > INT32_MAX)
        return hipErrorInvalidValue;
    const bool f64in = (mode == TDS_F64);
    const int32_t* own64 = own_items + items32;
    // a phase of two launches: its start event on the first, its stop on
    // the second
    KTime t1[3], t2[3];
    const KTime* p1[3] = {nullptr, nullptr, nullptr};
    const KTime* p2[3] = {nullptr, nullptr, nullptr};
    if (tm) {
        for (int q = 0; q < 3; ++q) {
            if (items32 > 0 && items64 > 0 && q != 1) {
                t1[q] = KTime{tm[q].start, nullptr};
                t2[q] = KTime{nullptr, tm[q].stop};
                p1[q] = &t1[q];
                p2[q] = &t2[q];
            } else {
                p1[q] = p2[q] = &tm[q];
            }
        }
    }
    if (items32 > 0) {
        const dim3 g((unsigned)items32);
        if (f64in)
            launch_k(k_beta_batch<32, double>, g, dim3(kWG), 0, s, p1[0], D, own_items);
        else
            launch_k(k_beta_batch<32, float>, g, dim3(kWG), 0, s, p1[0], D, own_items);
    }
    if (items64 > 0) {
        const dim3 g((unsigned)items64);
        if (f64in)
            launch_k(k_beta_batch<64, double>, g, dim3(kWG), 0, s, p2[0], D, own64);
        else
            launch_k(k_beta_batch<64, float>, g, dim3(kWG), 0, s, p2[0], D, own64);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (scans > 0) {
        launch_k(k_iface_batch, dim3((unsigned)scans), dim3(kScanBatchWide), 0, s, p1[1], D,
                 own_scans);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (items32 > 0) batch_sweep<32>(D, own_items, items32, mode, passes, false, s, p1[2]);
    if (items64 > 0) batch_sweep<64>(D, own64, items64, mode, passes, halves, s, p2[2]);
    return hipGetLastError();
}

int64_t fused_batch_sync_ints(int64_t S) { return kSyncStride * (2 + 2 * S); }


hipError_t launch_fused_batch(const BatchDesc* D, const uint64_t* tk, int64_t nitems, int64_t S,
                              int mode, int passes, int* sync, hipStream_t s, const KTime* tm) {
    if (nitems == 0) return hipSuccess;
    if (nitems > INT32_MAX || !sync || !tk) return hipErrorInvalidValue;
    const int64_t nsync = fused_batch_sync_ints(S);
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((nsync + kWG - 1) / kWG)), dim3(kWG), 0, s,
                       sync, nsync);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g((unsigned)((nitems + kFusedGroup - 1) / kFusedGroup));
    switch (mode) {
        case TDS_F64:
            launch_k(k_fused_batch<double, double, kSweep64>, g, dim3(kWG), 0, s, tm, D, tk,
                     nitems, S, passes, sync);
            break;
        case TDS_F32_WIDE:
            launch_k(k_fused_batch<float, double, kSweep64>, g, dim3(kWG), 0, s, tm, D, tk,
                     nitems, S, passes, sync);
            break;
        case TDS_F32:
            launch_k(k_fused_batch<float, float, kSweep32>, g, dim3(kWG), 0, s, tm, D, tk,
                     nitems, S, passes, sync);
            break;
        default:
            launch_k(k_fused_batch<float, double, kSweepRefined>, g, dim3(kWG), 0, s, tm, D, tk,
                     nitems, S, passes, sync);
            break;
    }
    return hipGetLastError();
}

}  // namespace tds
