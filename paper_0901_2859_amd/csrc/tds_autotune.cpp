// Measured choice of the block decomposition (number of blocks P, hence
// rows per block) for one matrix or for an uneven batch, and of the launch
// configuration and refinement passes of a plan.
//
// The split into P blocks is a free parameter of the method (Algorithm 3
// works for any P with blocks of at least 2 rows); it trades the
// per-right-hand-side interface work, which grows with P, against the block
// sweeps, whose register footprint grows with the rows per block.  Which
// balance is fastest depends on M, N, the mode and the device, so the
// candidates are simply timed: each one is prepared, solved on
// uniform[-1, 1) right-hand sides of the caller's N (generated on the
// device, or the caller's own), and the fastest is returned.  The number of
// refinement passes is chosen by accuracy, not speed: the fewest passes
// whose residual on the same right-hand sides stays within kPassesSlack
// times that of the solve in FP64 arithmetic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "tdsolve.h"
#include "tds_internal.h"

namespace {

using namespace tds;

// refined solves count as reaching the FP64 residual within this factor of
// the same plan's FP64-arithmetic solve (TDS_F32_WIDE)
constexpr double kPassesSlack = 1.25;

size_t f_bytes(int32_t mode) { return mode == TDS_F64 ? 8 : 4; }
size_t x_bytes(int32_t mode) { return mode == TDS_F32 ? 4 : 8; }

// block count with blocks of at most `rows` rows, within the method's limits
int32_t blocks_for(int64_t M, int32_t rows) {
    if (M < 4) return 1;
    int64_t P = (M + rows - 1) / rows;
    P = std::max<int64_t>(1, std::min<int64_t>(P, M / 2));
    return (int32_t)std::min<int64_t>(P, 65535);
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// average milliseconds per call of `run` (after two untimed calls)
template <typename Run>
int time_calls(Run run, int32_t reps, hipStream_t s, Events& ev, double* ms) {
    for (int w = 0; w < 2; ++w) {
        const int rc = run();
        if (rc) return rc;
    }
    if (hipEventRecord(ev.a, s) != hipSuccess) return TDS_EHIP;
    for (int r = 0; r < reps; ++r) {
        const int rc = run();
        if (rc) return rc;
    }
    if (hipEventRecord(ev.b, s) != hipSuccess) return TDS_EHIP;
    if (hipEventSynchronize(ev.b) != hipSuccess) return TDS_EHIP;
    float el = 0.f;
    if (hipEventElapsedTime(&el, ev.a, ev.b) != hipSuccess) return TDS_EHIP;
    *ms = (double)el / reps;
    return TDS_OK;
}

// Candidates are timed in interleaved rounds (every candidate once per
// round) and each keeps its fastest round: a candidate timed first would
// otherwise also pay for the device still raising its clocks.
constexpr int kRounds = 3;
// the fused order's candidate configuration (lag, tile)
constexpr int32_t kTuneLag = 8;
constexpr int32_t kTuneTile = 512;

int alloc(DevBuf& b, size_t bytes) {
    const hipError_t e = hipMalloc(&b.p, std::max<size_t>(bytes, 256));
    if (e == hipErrorOutOfMemory) return TDS_ENOMEM;
    return e == hipSuccess ? TDS_OK : TDS_EHIP;
}

// largest relative 2-norm residual of the series in X (tdsolve_residual)
int max_r2(tds_handle h, const void* F, const void* X, int64_t N, int32_t mode, double* out_dev,
           hipStream_t s, double* r2) {
    int rc = tdsolve_residual(h, F, X, N, mode, out_dev, s);
    if (rc) return rc;
    std::vector<double> host(2 * (size_t)N);
    if (hipMemcpyAsync(host.data(), out_dev, sizeof(double) * host.size(), hipMemcpyDeviceToHost,
                       s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return TDS_EHIP;
    double m = 0.0;
    for (int64_t n = 0; n < N; ++n) m = std::max(m, host[N + n]);
    *r2 = m;
    return TDS_OK;
}

}  // namespace

extern "C" {

int tdsolve_autotune(const double* a, const double* b, int64_t M, int64_t N, int32_t mode,
                     int32_t reps, int32_t* P_out, double* ms_out, void* stream) {
    if (!P_out || M < 1 || N < 1 || mode < TDS_F64 || mode > TDS_F32_WIDE) return TDS_EINVAL;
    if (reps <= 0) reps = 5;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> cand;
    for (int32_t rows : {16, 32, 64, 128}) cand.push_back(blocks_for(M, rows));
    if (M <= 128) cand.push_back(1);
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());

    DevBuf F, X;
    int rc = alloc(F, f_bytes(mode) * (size_t)M * (size_t)N);
    if (!rc) rc = alloc(X, x_bytes(mode) * (size_t)M * (size_t)N);
    if (rc) return rc;
    if (launch_fill_uniform(F.p, M * N, mode != TDS_F64, 0x5eedull, s) != hipSuccess)
        return TDS_EHIP;
    Events ev;
    if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess)
        return TDS_EHIP;
    std::vector<tds_handle> hs(cand.size(), nullptr);
    std::vector<double> best_ms(cand.size(), INFINITY);
    for (size_t c = 0; c < cand.size() && !rc; ++c) rc = tdsolve_prepare(a, b, M, cand[c], &hs[c]);
    for (int round = 0; round < kRounds && !rc; ++round)
        for (size_t c = 0; c < cand.size() && !rc; ++c) {
            double ms = 0.0;
            rc = time_calls([&] { return tdsolve_series(hs[c], F.p, X.p, N, mode, stream); }, reps,
                            s, ev, &ms);
            best_ms[c] = std::min(best_ms[c], ms);
        }
    for (tds_handle h : hs)
        if (h) tdsolve_destroy(h);
    if (rc) return rc;
    const size_t pick = std::min_element(best_ms.begin(), best_ms.end()) - best_ms.begin();
    *P_out = cand[pick];
    if (ms_out) *ms_out = best_ms[pick];
    return TDS_OK;
}

int tdsolve_autotune_plan(const double* a, const double* b, int64_t M, int64_t N, int32_t mode,
                          int32_t P, const void* Fin, int32_t reps, tds_tuning* out,
                          void* stream) {
    if (!out || M < 1 || N < 1 || P < 0 || mode < TDS_F64 || mode > TDS_F32_WIDE)
        return TDS_EINVAL;
    if (reps <= 0) reps = 5;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> cand;
    if (P > 0) {
        cand.push_back(P);
    } else {
        for (int32_t rows : {16, 32, 64, 128}) cand.push_back(blocks_for(M, rows));
        if (M <= 128) cand.push_back(1);
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    }
    DevBuf Fbuf, X, Xw, R;
    int rc = TDS_OK;
    const void* F = Fin;
    if (!F) {
        rc = alloc(Fbuf, f_bytes(mode) * (size_t)M * (size_t)N);
        if (rc) return rc;
        if (launch_fill_uniform(Fbuf.p, M * N, mode != TDS_F64, 0x5eedull, s) != hipSuccess)
            return TDS_EHIP;
        F = Fbuf.p;
    }
    rc = alloc(X, x_bytes(mode) * (size_t)M * (size_t)N);
    if (!rc && mode == TDS_F32_REFINED) rc = alloc(Xw, sizeof(double) * (size_t)M * (size_t)N);
    if (!rc) rc = alloc(R, sizeof(double) * 2 * (size_t)N);
    if (rc) return rc;
    Events ev;
    if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess)
        return TDS_EHIP;

    // one plan per block count; its refinement passes first (the fewest,
    // 1..3, whose largest relative residual on these right-hand sides stays
    // within kPassesSlack times that of the same solve in FP64 arithmetic),
    // then the launch configurations timed under them
    struct Cand {
        size_t plan;
        int32_t order, lag, tile;
        double ms = INFINITY;
    };
    std::vector<tds_handle> hs(cand.size(), nullptr);
    std::vector<int32_t> passes(cand.size(), 0);
    std::vector<double> r2s(cand.size(), 0.0);
    std::vector<Cand> cs;
    for (size_t c = 0; c < cand.size() && !rc; ++c) {
        rc = tdsolve_prepare(a, b, M, cand[c], &hs[c]);
        if (rc) break;
        tds_info info;
        tdsolve_info(hs[c], &info);
        if (mode == TDS_F32_REFINED) {
            double r2w = 0.0;
            rc = tdsolve_series(hs[c], F, Xw.p, N, TDS_F32_WIDE, stream);
            if (!rc) rc = max_r2(hs[c], F, Xw.p, N, TDS_F32_WIDE, (double*)R.p, s, &r2w);
            int32_t p = 1;
            for (; !rc && p <= 3; ++p) {
                double r2 = 0.0;
                rc = tdsolve_set_refinement(hs[c], p);
                if (!rc) rc = tdsolve_series(hs[c], F, X.p, N, mode, stream);
                if (!rc) rc = max_r2(hs[c], F, X.p, N, mode, (double*)R.p, s, &r2);
                r2s[c] = r2;
                if (!rc && r2 <= kPassesSlack * r2w) break;
            }
            passes[c] = std::min<int32_t>(p, 3);
            if (!rc) rc = tdsolve_set_refinement(hs[c], passes[c]);
        }
        const bool dense_ok = cand[c] >= 2 && cand[c] <= kDenseMaxBlocks;
        for (int32_t order : {TDS_IFACE_RECURRENCE, TDS_IFACE_DENSE}) {
            if (order == TDS_IFACE_DENSE && !dense_ok) continue;
            cs.push_back({c, order, 0, 0});
            if (info.sweep_halves && mode != TDS_F32) cs.push_back({c, order, kTuneLag, kTuneTile});
        }
    }
    for (int round = 0; round < kRounds && !rc; ++round)
        for (Cand& k : cs) {
            tds_handle h = hs[k.plan];
            rc = tdsolve_set_interface(h, k.order);
            if (!rc) rc = tdsolve_set_fused(h, k.lag, k.tile);
            if (rc) break;
            double ms = 0.0;
            rc = time_calls([&] { return tdsolve_series(h, F, X.p, N, mode, stream); }, reps, s,
                            ev, &ms);
            k.ms = std::min(k.ms, ms);
        }
    if (!rc && !cs.empty()) {
        const Cand& k = *std::min_element(cs.begin(), cs.end(),
                                          [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
        out->P = cand[k.plan];
        out->order = k.order;
        out->passes = passes[k.plan];
        out->fuse_lag = k.lag;
        out->fuse_tile = k.tile;
        out->ms = k.ms;
        // the residual of the chosen configuration
        tds_handle h = hs[k.plan];
        rc = tdsolve_set_interface(h, k.order);
        if (!rc) rc = tdsolve_set_fused(h, k.lag, k.tile);
        if (!rc) rc = tdsolve_series(h, F, X.p, N, mode, stream);
        if (!rc) rc = max_r2(h, F, X.p, N, mode, (double*)R.p, s, &out->r2);
    }
    for (tds_handle h : hs)
        if (h) tdsolve_destroy(h);
    return rc;
}

int tdsolve_batch_autotune(int32_t K, const double* const* a, const double* const* b,
                           const int64_t* M, const int64_t* N, int32_t mode, int32_t reps,
                           int32_t* P_out, int32_t* passes_out, int32_t* lag_out,
                           double* ms_out, void* stream) {
    if (K < 1 || !a || !b || !M || !N || !P_out || mode < TDS_F64 || mode > TDS_F32_WIDE)
        return TDS_EINVAL;
    if (reps <= 0) reps = 5;
    hipStream_t s = (hipStream_t)stream;
    // one buffer for every matrix's F and X, 256-byte aligned slices
    std::vector<size_t> fo(K), xo(K);
    size_t fb = 0, xb = 0;
    for (int32_t k = 0; k < K; ++k) {
        if (M[k] < 1 || N[k] < 0) return TDS_EINVAL;
        fo[k] = fb;
        xo[k] = xb;
        fb += (f_bytes(mode) * (size_t)M[k] * (size_t)N[k] + 255) / 256 * 256;
        xb += (x_bytes(mode) * (size_t)M[k] * (size_t)N[k] + 255) / 256 * 256;
    }
    DevBuf F, X;
    int rc = alloc(F, fb);
    if (!rc) rc = alloc(X, xb);
    if (rc) return rc;
    const size_t fe = f_bytes(mode);
    if (launch_fill_uniform(F.p, (int64_t)(fb / fe), mode != TDS_F64, 0x5eedull, s) !=
        hipSuccess)
        return TDS_EHIP;
    std::vector<const void*> Fp(K);
    std::vector<void*> Xp(K);
    for (int32_t k = 0; k < K; ++k) {
        Fp[k] = (const unsigned char*)F.p + fo[k];
        Xp[k] = (unsigned char*)X.p + xo[k];
    }
    Events ev;
    if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess)
        return TDS_EHIP;
    // rows per block, 32 or 64 (the batch runs one launch of each kernel per
    // register row bucket): first the same for every matrix
    const int32_t rows_c[2] = {32, 64};
    tds_handle hs[2] = {nullptr, nullptr};
    std::vector<int32_t> P(K);
    double best_ms[2] = {INFINITY, INFINITY};
    for (int c = 0; c < 2 && !rc; ++c) {
        for (int32_t k = 0; k < K; ++k) P[k] = blocks_for(M[k], rows_c[c]);
        rc = tdsolve_batch_prepare(K, a, b, M, P.data(), &hs[c]);
    }
    auto series = [&](tds_handle h) {
        return tdsolve_batch_series(h, Fp.data(), Xp.data(), N, mode, stream);
    };
    for (int round = 0; round < kRounds && !rc; ++round)
        for (int c = 0; c < 2 && !rc; ++c) {
            double ms = 0.0;
            rc = time_calls([&] { return series(hs[c]); }, reps, s, ev, &ms);
            best_ms[c] = std::min(best_ms[c], ms);
        }
    const int uni = best_ms[1] < best_ms[0] ? 1 : 0;
    tds_handle cur = hs[uni];
    if (hs[1 - uni]) tdsolve_destroy(hs[1 - uni]);
    hs[0] = hs[1] = nullptr;
    double cur_ms = best_ms[uni];
    std::vector<int32_t> rows(K, rows_c[uni]);
    // then per matrix: the matrices in four classes of equal count by size
    // (M[k] N[k]); from the uniform choice, each class's rows per block are
    // flipped in turn, largest class first, and kept when the batch is
    // faster (the current and the flipped batch timed in alternation)
    std::vector<int32_t> order(K);
    for (int32_t k = 0; k < K; ++k) order[k] = k;
    std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return (double)M[x] * (double)N[x] < (double)M[y] * (double)N[y];
    });
    const int32_t classes = K >= 4 ? 4 : 1;
    for (int32_t c = classes - 1; c >= 0 && !rc; --c) {
        const int32_t k0 = (int32_t)((int64_t)K * c / classes);
        const int32_t k1 = (int32_t)((int64_t)K * (c + 1) / classes);
        std::vector<int32_t> trial(rows);
        for (int32_t i = k0; i < k1; ++i) trial[order[i]] = trial[order[i]] == 32 ? 64 : 32;
        for (int32_t k = 0; k < K; ++k) P[k] = blocks_for(M[k], trial[k]);
        tds_handle th = nullptr;
        rc = tdsolve_batch_prepare(K, a, b, M, P.data(), &th);
        double t_cur = INFINITY, t_try = INFINITY;
        for (int round = 0; round < kRounds && !rc; ++round) {
            double ms = 0.0;
            rc = time_calls([&] { return series(cur); }, reps, s, ev, &ms);
            t_cur = std::min(t_cur, ms);
            if (!rc) rc = time_calls([&] { return series(th); }, reps, s, ev, &ms);
            t_try = std::min(t_try, ms);
        }
        if (!rc && t_try < t_cur) {
            tdsolve_destroy(cur);
            cur = th;
            rows = trial;
            cur_ms = t_try;
        } else {
            if (th) tdsolve_destroy(th);
            if (!rc) cur_ms = std::min(cur_ms, t_cur);
        }
    }
    // refinement passes: the fewest (1..3) whose largest normwise backward
    // error on these right-hand sides stays within kPassesSlack times that
    // of the same solve in FP64 arithmetic (TDS_F32_WIDE)
    int32_t passes = 0;
    if (!rc && mode == TDS_F32_REFINED) {
        double eta_wide = 0.0;
        rc = tdsolve_batch_series(cur, Fp.data(), Xp.data(), N, TDS_F32_WIDE, stream);
        if (!rc) rc = tdsolve_status(cur, stream, &eta_wide, nullptr);
        for (passes = 1; !rc && passes <= 3; ++passes) {
            double eta = 0.0;
            rc = tdsolve_set_refinement(cur, passes);
            if (!rc) rc = series(cur);
            if (!rc) rc = tdsolve_status(cur, stream, &eta, nullptr);
            if (!rc && eta <= kPassesSlack * eta_wide) break;
        }
        if (passes > 3) passes = 3;
    }
    // launch order: the one-launch order (tdsolve_batch_set_fused) at a few
    // lags, with every matrix in the 32-row bucket, against the chosen
    // blocks in separate launches, in interleaved rounds.  When the chosen
    // blocks are not all 32-row ones, the one launch runs on 32-row blocks
    // of its own (not for the refined mode, whose passes were chosen for
    // the chosen blocks).  On the 256-matrix benchmark batch the one launch
    // runs best at a lag of 16 tiles and is faster than the separate
    // launches in FP64 arithmetic, slower for the refined mode.
    int32_t lag = 0;
    bool all32 = true;
    for (int32_t k = 0; k < K; ++k) all32 = all32 && rows[k] == 32;
    if (!rc && (all32 || mode != TDS_F32_REFINED)) {
        tds_handle h32 = all32 ? cur : nullptr;
        if (!all32) {
            for (int32_t k = 0; k < K; ++k) P[k] = blocks_for(M[k], 32);
            rc = tdsolve_batch_prepare(K, a, b, M, P.data(), &h32);
        }
        const int32_t lags[4] = {0, 8, 16, 32};
        double t_lag[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
        double t_cur = INFINITY;
        for (int round = 0; round < kRounds && !rc; ++round) {
            double ms = 0.0;
            if (!all32) {
                rc = time_calls([&] { return series(cur); }, reps, s, ev, &ms);
                t_cur = std::min(t_cur, ms);
            }
            for (int i = all32 ? 0 : 1; i < 4 && !rc; ++i) {
                rc = tdsolve_batch_set_fused(h32, lags[i]);
                if (!rc) rc = series(h32);          // uploads the ticket table
                if (!rc) rc = time_calls([&] { return series(h32); }, reps, s, ev, &ms);
                t_lag[i] = std::min(t_lag[i], ms);
            }
        }
        if (all32) t_cur = t_lag[0];
        int best = 0;
        for (int i = 1; i < 4; ++i)
            if (t_lag[i] < (best ? t_lag[best] : t_cur)) best = i;
        if (!rc) {
            if (best > 0) {
                lag = lags[best];
                cur_ms = t_lag[best];
                for (int32_t k = 0; k < K; ++k) rows[k] = 32;
            } else {
                cur_ms = t_cur;
            }
        }
        if (h32 && h32 != cur) tdsolve_destroy(h32);
    }
    if (cur) tdsolve_destroy(cur);
    if (rc) return rc;
    for (int32_t k = 0; k < K; ++k) P_out[k] = blocks_for(M[k], rows[k]);
    if (passes_out) *passes_out = passes;
    if (lag_out) *lag_out = lag;
    if (ms_out) *ms_out = cur_ms;
    return TDS_OK;
}

}  // extern "C"
