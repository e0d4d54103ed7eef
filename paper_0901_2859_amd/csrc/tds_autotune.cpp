// Measured choice of the block decomposition (number of blocks P, hence
// rows per block) for one matrix or for an uneven batch.
//
// The split into P blocks is a free parameter of the method (Algorithm 3
// works for any P with blocks of at least 2 rows); it trades the
// per-right-hand-side interface work, which grows with P, against the block
// sweeps, whose register footprint grows with the rows per block.  Which
// balance is fastest depends on M, N, the mode and the device, so the
// candidates are simply timed: each one is prepared, solved on
// uniform[-1, 1) right-hand sides of the caller's N (generated on the
// device), and the fastest is returned.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "tdsolve.h"
#include "tds_internal.h"

namespace {

using namespace tds;

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

int alloc(DevBuf& b, size_t bytes) {
    const hipError_t e = hipMalloc(&b.p, std::max<size_t>(bytes, 256));
    if (e == hipErrorOutOfMemory) return TDS_ENOMEM;
    return e == hipSuccess ? TDS_OK : TDS_EHIP;
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
    double best = INFINITY;
    int32_t bestP = 0;
    for (int32_t P : cand) {
        tds_handle h = nullptr;
        rc = tdsolve_prepare(a, b, M, P, &h);
        if (rc) return rc;
        double ms = 0.0;
        rc = time_calls([&] { return tdsolve_series(h, F.p, X.p, N, mode, stream); }, reps, s,
                        ev, &ms);
        tdsolve_destroy(h);
        if (rc) return rc;
        if (ms < best) {
            best = ms;
            bestP = P;
        }
    }
    *P_out = bestP;
    if (ms_out) *ms_out = best;
    return TDS_OK;
}

int tdsolve_batch_autotune(int32_t K, const double* const* a, const double* const* b,
                           const int64_t* M, const int64_t* N, int32_t mode, int32_t reps,
                           int32_t* P_out, double* ms_out, void* stream) {
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
    // the batch kernels share one register row bucket: 32 or 64 rows
    double best = INFINITY;
    int32_t best_rows = 0;
    std::vector<int32_t> P(K);
    for (int32_t rows : {32, 64}) {
        for (int32_t k = 0; k < K; ++k) P[k] = blocks_for(M[k], rows);
        tds_handle h = nullptr;
        rc = tdsolve_batch_prepare(K, a, b, M, P.data(), &h);
        if (rc) return rc;
        double ms = 0.0;
        rc = time_calls(
            [&] { return tdsolve_batch_series(h, Fp.data(), Xp.data(), N, mode, stream); }, reps,
            s, ev, &ms);
        tdsolve_destroy(h);
        if (rc) return rc;
        if (ms < best) {
            best = ms;
            best_rows = rows;
        }
    }
    for (int32_t k = 0; k < K; ++k) P_out[k] = blocks_for(M[k], best_rows);
    if (ms_out) *ms_out = best;
    return TDS_OK;
}

}  // extern "C"
