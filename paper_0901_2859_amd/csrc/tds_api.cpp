// C ABI of the tdsolve library (declared in include/tdsolve.h): argument
// checks, device tables of the preliminary step, work buffers and the
// launch sequence of the per-right-hand-side step.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "tdsolve.h"
#include "tds_internal.h"

using namespace tds;

struct tds_plan {
    HostTables host;
    DevTables dev;
    // half-block tables (half_tables) of the sweeps with FP64 results, when
    // the blocks fit them
    bool has_halves = false;
    DevTables halves;
    void* dev_mem = nullptr;
    double normA = 0.0;          // ||A||_inf
    int32_t passes = 2;          // refinement passes of TDS_F32_REFINED
    int32_t iface = TDS_IFACE_RECURRENCE;   // interface-step evaluation order
    double* dense_K = nullptr;   // Theorem 2 coefficient table (TDS_IFACE_DENSE)
    int32_t dense_Pc = 0, dense_Mr = 0;
    int32_t fuse_lag = 0;        // fused order: interface items this many tiles behind the
                                 //   weights, sweeps twice that (0: separate kernels)
    int32_t fuse_cols = 0;       // fused order: right-hand sides per tile
    int device = 0;
    void* work = nullptr;        // grows with N
    size_t work_bytes = 0;
    bool timing = false;         // record per-phase events
    std::vector<hipEvent_t> events;  // per timed call: start, stop of beta, interface, sweep
    std::vector<uint8_t> timed_empty;    // per timed call: bit k = phase k launched nothing
    size_t events_used = 0;
    // batch handles: K matrices sharing one table allocation
    bool is_batch = false;
    std::vector<int32_t> buckets;        // register-sweep row bucket (32, 64) of each matrix
    std::vector<HostTables> hosts;
    std::vector<DevTables> devs;
    std::vector<DevTables> devs_h;       // half-block tables of the 64-row matrices, when
                                         //   every one of them has them
    std::vector<BatchDesc> desc;         // last descriptors uploaded
    BatchDesc* d_desc = nullptr;         // descriptors, then the item owner maps and
                                         //   the one-launch order's ticket table
    size_t desc_bytes = 0;               // capacity of d_desc
    int32_t desc_lag = 0;                // one-launch lag the uploaded ticket table is for
    // the last series call, for tdsolve_status
    bool have_last = false;
    int32_t last_mode = 0, last_passes = 0;
    std::vector<const void*> last_F;
    std::vector<const void*> last_X;
    std::vector<int64_t> last_N;
};

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Append one matrix's device tables to a host image; the returned tables
// hold byte offsets into the image in place of pointers (see rebase()).
// Row tables carry kRegMaxRows + 1 padding rows (a = cp = 0, b = rd = 1) so
// that the register sweep's phantom rows always read in bounds.  `WP` is
// the row count the per-block beta weights are zero-padded to (0: none).
DevTables append_image(const HostTables& o, int32_t WP, std::vector<unsigned char>& img) {
    const int64_t M = o.M;
    const int32_t P = o.P;
    const int64_t MR = M + kRegMaxRows + 1;
    size_t off = align256(img.size());
    auto take = [&](size_t bytes) { size_t at = off; off = align256(off + bytes); return at; };
    const size_t o_starts = take(sizeof(int64_t) * (P + 1));
    const size_t o_wR = take(sizeof(double) * MR), o_wL = take(sizeof(double) * MR);
    const size_t o_rho = take(sizeof(double) * P), o_lam = take(sizeof(double) * P);
    const size_t o_a64 = take(sizeof(double) * MR), o_b64 = take(sizeof(double) * MR);
    const size_t o_l64 = take(sizeof(double) * MR), o_inl64 = take(sizeof(double) * MR);
    const size_t o_l32 = take(sizeof(float) * MR), o_inl32 = take(sizeof(float) * MR);
    const size_t o_cp64 = take(sizeof(double) * MR), o_rd64 = take(sizeof(double) * MR);
    const size_t o_wpad = take(sizeof(double) * 2 * (size_t)P * (size_t)(WP > 0 ? WP : 1));
    const size_t o_in64 = take(sizeof(double) * MR), o_u = take(sizeof(double) * MR);
    const size_t o_v = take(sizeof(double) * MR);
    const size_t o_a32 = take(sizeof(float) * MR), o_cp32 = take(sizeof(float) * MR);
    const size_t o_rd32 = take(sizeof(float) * MR), o_in32 = take(sizeof(float) * MR);
    const size_t o_mid = take(sizeof(double) * P);
    const size_t o_eR = take(sizeof(float) * MR);
    const size_t nslot = std::max<size_t>(o.tw_r.size(), 1);
    const size_t o_tws = take(sizeof(double) * nslot), o_twr = take(sizeof(double) * nslot);
    const size_t o_twc = take(sizeof(double) * nslot), o_twe = take(sizeof(double) * nslot);
    img.resize(off, 0);

    auto put = [&](size_t at, const void* src, size_t bytes) { memcpy(img.data() + at, src, bytes); };
    auto pad64 = [&](size_t at, const std::vector<double>& v, double fill) {
        std::vector<double> t(v.begin(), v.end());
        t.resize(MR, fill);
        put(at, t.data(), sizeof(double) * MR);
    };
    auto pad32 = [&](size_t at, const std::vector<double>& v, float fill) {
        std::vector<float> t(MR, fill);
        for (int64_t i = 0; i < M; ++i) t[i] = (float)v[i];
        put(at, t.data(), sizeof(float) * MR);
    };
    put(o_starts, o.starts.data(), sizeof(int64_t) * (P + 1));
    pad64(o_wR, o.wR, 0.0);
    pad64(o_wL, o.wL, 0.0);
    put(o_rho, o.rho.data(), sizeof(double) * P);
    put(o_lam, o.lam.data(), sizeof(double) * P);
    pad64(o_a64, o.a64, 0.0);
    pad64(o_b64, o.b64, 1.0);
    pad64(o_cp64, o.cp64, 0.0);
    pad64(o_rd64, o.rd64, 1.0);
    if (WP > 0) {
        // beta weights of every block, zero-padded to the register kernel's
        // row count, so that rows past a block's end weigh nothing
        std::vector<double> wp(2 * (size_t)P * WP, 0.0);
        for (int32_t j = 0; j < P; ++j)
            for (int64_t i = o.starts[j]; i < o.starts[j + 1]; ++i) {
                const size_t r = (size_t)j * WP + (size_t)(i - o.starts[j]);
                wp[2 * r] = o.wR[i];
                wp[2 * r + 1] = o.wL[i];
            }
        put(o_wpad, wp.data(), sizeof(double) * wp.size());
    }
    std::vector<double> in(o.a64), inl(o.l64);
    for (int32_t j = 0; j < P; ++j) {                                 // block ends
        in[o.starts[j + 1] - 1] = 0.0;
        inl[o.starts[j + 1] - 1] = 0.0;
    }
    pad64(o_in64, in, 0.0);
    pad64(o_l64, o.l64, 0.0);
    pad64(o_inl64, inl, 0.0);
    pad32(o_l32, o.l64, 0.0f);
    pad32(o_inl32, inl, 0.0f);
    pad64(o_u, o.u, 0.0);
    pad64(o_v, o.v, 0.0);
    pad32(o_a32, o.a64, 0.0f);
    pad32(o_cp32, o.cp64, 0.0f);
    pad32(o_rd32, o.rd64, 1.0f);
    pad32(o_in32, in, 0.0f);
    if (!o.mid_inv.empty()) put(o_mid, o.mid_inv.data(), sizeof(double) * P);
    if (!o.eR.empty()) pad32(o_eR, o.eR, 0.0f);
    if (!o.tw_r.empty()) {
        put(o_tws, o.tw_s.data(), sizeof(double) * nslot);
        put(o_twr, o.tw_r.data(), sizeof(double) * nslot);
        put(o_twc, o.tw_c.data(), sizeof(double) * nslot);
        put(o_twe, o.tw_e.data(), sizeof(double) * nslot);
    }

    DevTables d;
    d.M = M;
    d.P = P;
    d.max_rows = o.max_rows;
    d.starts = (int64_t*)o_starts;
    d.wR = (double*)o_wR;
    d.wL = (double*)o_wL;
    d.rho = (double*)o_rho;
    d.lam = (double*)o_lam;
    d.general = o.general;
    d.a64 = (double*)o_a64;
    d.l64 = (double*)o_l64;
    d.inl64 = (double*)o_inl64;
    d.l32 = (float*)o_l32;
    d.inl32 = (float*)o_inl32;
    d.b64 = (double*)o_b64;
    d.cp64 = (double*)o_cp64;
    d.rd64 = (double*)o_rd64;
    d.wpad = (const double2*)o_wpad;
    d.wpad_rows = WP;
    d.in64 = (double*)o_in64;
    d.u = (double*)o_u;
    d.v = (double*)o_v;
    d.a32 = (float*)o_a32;
    d.cp32 = (float*)o_cp32;
    d.rd32 = (float*)o_rd32;
    d.in32 = (float*)o_in32;
    d.mid_inv = (double*)o_mid;
    d.eR32 = (float*)o_eR;
    d.tw_s = (double*)o_tws;
    d.tw_c = (double*)o_twc;
    d.tw_r = (double*)o_twr;
    d.tw_e = (double*)o_twe;
    return d;
}

template <typename T>
void shift(T*& p, unsigned char* base) { p = (T*)(base + (size_t)p); }
template <typename T>
void shift(const T*& p, unsigned char* base) { p = (const T*)(base + (size_t)p); }

void rebase(DevTables& d, void* mem) {
    unsigned char* b = (unsigned char*)mem;
    shift(d.starts, b); shift(d.wR, b); shift(d.wL, b); shift(d.rho, b); shift(d.lam, b);
    shift(d.a64, b); shift(d.b64, b); shift(d.cp64, b); shift(d.rd64, b); shift(d.wpad, b);
    shift(d.in64, b); shift(d.u, b); shift(d.v, b); shift(d.a32, b); shift(d.cp32, b);
    shift(d.rd32, b); shift(d.in32, b);
    shift(d.l64, b); shift(d.inl64, b); shift(d.l32, b); shift(d.inl32, b);
    shift(d.mid_inv, b);
    shift(d.eR32, b); shift(d.tw_s, b); shift(d.tw_c, b); shift(d.tw_r, b); shift(d.tw_e, b);
}

int upload_image(const std::vector<unsigned char>& img, void** out) {
    void* mem = nullptr;
    hipError_t e = hipMalloc(&mem, std::max<size_t>(img.size(), 256));
    if (e == hipErrorOutOfMemory) return TDS_ENOMEM;
    if (e != hipSuccess) return TDS_EHIP;
    if (hipMemcpy(mem, img.data(), img.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(mem);
        return TDS_EHIP;
    }
    *out = mem;
    return TDS_OK;
}

int upload(tds_plan* h) {
    if (hipGetDevice(&h->device) != hipSuccess) return TDS_EHIP;
    std::vector<unsigned char> img;
    h->dev = append_image(h->host, rows_bucket(h->host.max_rows), img);
    // blocks of 35..64 rows: the sweeps with FP64 results take them in halves
    HostTables hh;
    h->has_halves = rows_bucket(h->host.max_rows) == 64 &&
                    half_tables(h->host, kHalfRows, hh) == TDS_OK;
    if (h->has_halves) h->halves = append_image(hh, 0, img);
    int rc = upload_image(img, &h->dev_mem);
    if (rc) return rc;
    rebase(h->dev, h->dev_mem);
    if (h->has_halves) rebase(h->halves, h->dev_mem);
    return TDS_OK;
}

int ensure_work(tds_plan* h, size_t bytes) {
    if (bytes <= h->work_bytes) return TDS_OK;
    if (h->work) {
        // the previous buffer may still be in use by queued work
        if (hipDeviceSynchronize() != hipSuccess) return TDS_EHIP;
        (void)hipFree(h->work);
        h->work = nullptr;
        h->work_bytes = 0;
    }
    hipError_t e = hipMalloc(&h->work, bytes);
    if (e == hipErrorOutOfMemory) return TDS_ENOMEM;
    if (e != hipSuccess) return TDS_EHIP;
    h->work_bytes = bytes;
    return TDS_OK;
}

char* general_of(tds_plan* h) { return (char*)h->work; }

bool valid_mode(int32_t m) { return m >= TDS_F64 && m <= TDS_F32_WIDE; }
size_t f_elem(int32_t m) { return m == TDS_F64 ? 8 : 4; }
size_t x_elem(int32_t m) { return m == TDS_F32 ? 4 : 8; }

int check_common(tds_plan* h, int64_t N, int32_t mode) {
    if (!h || h->is_batch) return TDS_EINVAL;
    if (N < 0 || !valid_mode(mode)) return TDS_EINVAL;
    // the narrowest workgroups take 16 right-hand sides (interface steps)
    if ((N + kScanRhs - 1) / kScanRhs > 0x7fffffffLL) return TDS_EUNSUPPORTED;
    return TDS_OK;
}

// Slices of the plan's work buffer for N right-hand sides: beta^R, beta^L
// (P x N), the interface values (P-1 x N) and, for the dichotomy, its two
// partial sums ((P+1) x N each).
struct Work {
    double* betaR;
    double* betaL;
    double* xsep;
    double* SR;
    double* SL;
    int* sync;       // counters of the fused order (fused_sync_ints(N))
};

// bytes of the work slices for N right-hand sides; nb, nx, ns: the slice sizes
size_t work_bytes(const tds_plan* h, int64_t N, size_t* nb_, size_t* nx_, size_t* ns_) {
    const size_t P = (size_t)h->dev.P;
    const size_t nb = align256(sizeof(double) * P * (size_t)N);
    const size_t nx = align256(sizeof(double) * (P > 1 ? P - 1 : 1) * (size_t)N);
    const size_t ns = (h->iface == TDS_IFACE_DICHOTOMY)
                          ? align256(sizeof(double) * (P + 1) * (size_t)N) : 0;
    const size_t nc = align256(sizeof(int) * (size_t)fused_sync_ints(N));
    if (nb_) *nb_ = nb;
    if (nx_) *nx_ = nx;
    if (ns_) *ns_ = ns;
    return 2 * nb + nx + 2 * ns + nc;
}

// the slices laid out from `base`
void carve_work(const tds_plan* h, int64_t N, char* base, Work& w) {
    size_t nb, nx, ns;
    (void)work_bytes(h, N, &nb, &nx, &ns);
    w.betaR = (double*)base;
    w.betaL = (double*)(base + nb);
    w.xsep = (double*)(base + 2 * nb);
    w.SR = ns ? (double*)(base + 2 * nb + nx) : nullptr;
    w.SL = ns ? (double*)(base + 2 * nb + nx + ns) : nullptr;
    w.sync = (int*)(base + 2 * nb + nx + 2 * ns);
}

int take_work(tds_plan* h, int64_t N, Work& w) {
    const int rc = ensure_work(h, work_bytes(h, N, nullptr, nullptr, nullptr));
    if (rc) return rc;
    carve_work(h, N, general_of(h), w);
    return TDS_OK;
}

// Theorem 2's interface values from the beta weights, in the plan's order
hipError_t run_iface(tds_plan* h, const Work& w, double* xsep, int64_t N, hipStream_t s,
                     const KTime* tm = nullptr) {
    if (h->iface == TDS_IFACE_DICHOTOMY)
        return launch_iface_dichotomy(h->dev, w.betaR, w.betaL, w.SR, w.SL, xsep, N, s, tm);
    if (h->iface == TDS_IFACE_DENSE)
        return launch_iface_dense(h->dense_K, h->dense_Pc, h->dense_Mr, h->dev.P, w.betaR,
                                  w.betaL, xsep, N, s, tm);
    return launch_iface(h->dev, w.betaR, w.betaL, xsep, N, s, tm);
}

constexpr size_t kTimedEvents = 6;   // start and stop of beta, interface, sweep

// the start/stop pairs of one timed call (null when timing is off); the
// events take the kernels' own start and end timestamps
KTime* timing_slot(tds_plan* h) {
    if (!h->timing) return nullptr;
    while (h->events.size() < h->events_used + kTimedEvents) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->events.push_back(e);
    }
    static_assert(sizeof(KTime) == 2 * sizeof(hipEvent_t), "KTime is a pair of events");
    KTime* tm = reinterpret_cast<KTime*>(h->events.data() + h->events_used);
    h->events_used += kTimedEvents;
    h->timed_empty.push_back(0);
    return tm;
}

// phase k of the current timed call launches no kernel: its events stay
// unrecorded and it reads as zero
void empty_phase(tds_plan* h, int k) { h->timed_empty.back() |= (uint8_t)(1u << k); }

// `given` (may be null): work slices supplied by the caller (the entry point
// that allocates nothing); then the call neither grows the plan's work
// buffer nor records phase timing
int series_impl(tds_plan* h, const void* F, void* X, int64_t N, int32_t mode, hipStream_t s,
                int sweep_mode, const Work* given = nullptr) {
    const DevTables& t = h->dev;
    Work w;
    if (given) {
        w = *given;
    } else {
        const int rc = take_work(h, N, w);
        if (rc) return rc;
    }
    double* xsep = w.xsep;
    KTime* tm = given ? nullptr : timing_slot(h);
    if (h->timing && !given && !tm) return TDS_EHIP;
    if (h->fuse_lag > 0 && fused_fits(t, h->has_halves ? &h->halves : nullptr, F, N,
                                      sweep_mode, h->iface)) {
        // the whole solve as one fused launch (timed as the sweep phase)
        if (tm) {
            empty_phase(h, 0);
            empty_phase(h, 1);
        }
        const bool dense = h->iface == TDS_IFACE_DENSE;
        if (launch_fused(t, h->halves, F, X, N, sweep_mode, h->passes, w.betaR, w.betaL, xsep,
                         dense ? h->dense_K : nullptr, h->dense_Pc, h->dense_Mr, h->fuse_lag,
                         h->fuse_cols, w.sync, s, tm ? tm + 2 : nullptr) != hipSuccess)
            return TDS_EHIP;
        return TDS_OK;
    }
    if (t.P >= 2 && N > 0) {
        if (launch_beta(t, F, mode != TDS_F64, N, w.betaR, w.betaL, s, tm) != hipSuccess)
            return TDS_EHIP;
        if (run_iface(h, w, xsep, N, s, tm ? tm + 1 : nullptr) != hipSuccess) return TDS_EHIP;
    } else if (tm) {
        empty_phase(h, 0);
        empty_phase(h, 1);
    }
    if (N > 0) {
        if (launch_sweep(t, F, X, N, sweep_mode, h->passes, xsep, s, tm ? tm + 2 : nullptr,
                         h->has_halves ? &h->halves : nullptr) != hipSuccess)
            return TDS_EHIP;
    } else if (tm) {
        empty_phase(h, 2);
    }
    return TDS_OK;
}

// zero fill by a kernel (not a memset node, so that captured graphs replay it
// reliably)
__global__ void k_zero_f64(double* __restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < n; k += stride) dst[k] = 0.0;
}

hipError_t zero_f64(double* p, int64_t n, hipStream_t s) {
    if (!p || n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_f64, dim3(blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// ||A||_inf from the host tables
double norm_inf(const HostTables& o) {
    double normA = 0.0;
    for (int64_t i = 0; i < o.M; ++i) {
        const double r = fabs(o.b64[i]) + (i > 0 ? fabs(o.l64[i - 1]) : 0.0) + fabs(o.a64[i]);
        normA = std::max(normA, r);
    }
    return normA;
}

// F and X of one solve may be the same array, but not partly overlap
bool overlap(const void* F, size_t fbytes, const void* X, size_t xbytes) {
    const uintptr_t f0 = (uintptr_t)F, x0 = (uintptr_t)X;
    return F != X && f0 < x0 + xbytes && x0 < f0 + fbytes;
}

void remember(tds_plan* h, const void* const* F, void* const* X, const int64_t* N, int32_t K,
              int32_t mode) {
    h->last_F.assign(F, F + K);
    h->last_X.assign(X, X + K);
    h->last_N.assign(N, N + K);
    h->last_mode = mode;
    h->last_passes = mode == TDS_F32_REFINED ? h->passes : 0;
    h->have_last = true;
}

// ---- fixed work area of tdsolve_series_noalloc ----------------------------
// The beta weights and interface values of that entry point live in this
// file-scope device array instead of the plan's growing work buffer.  Each
// GPU that loads the library holds its own copy for the life of the
// process.  Host code never passes the array's name to a kernel or a copy:
// its device address is taken once per device with hipGetSymbolAddress and
// kept in noalloc_base[].
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex noalloc_mu;
void* noalloc_base[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first
// call per device); TDS_OK or TDS_EHIP
int noalloc_scratch(int device, char** out) {
    if (device < 0 || device >= kMaxDevices) return TDS_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_base[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return TDS_EHIP;
        noalloc_base[device] = ptr;
    }
    *out = (char*)noalloc_base[device];
    return TDS_OK;
}

constexpr int32_t kFuseMaxLag = 64;

}  // namespace

extern "C" {

// checks, ||A||_inf and upload after the host tables are in place
static int finish_plan(tds_plan* h, tds_handle* out) {
    if (h->host.P > 65535) { delete h; return TDS_EUNSUPPORTED; }
    h->normA = norm_inf(h->host);
    const int rc = upload(h);
    if (rc) { delete h; return rc; }
    *out = h;
    return TDS_OK;
}

int tdsolve_prepare(const double* a, const double* b, int64_t M, int32_t P, tds_handle* out) {
    if (!out) return TDS_EINVAL;
    *out = nullptr;
    tds_plan* h = new (std::nothrow) tds_plan();
    if (!h) return TDS_ENOMEM;
    int rc = host_prepare(a, b, M, P, h->host);
    if (rc) { delete h; return rc; }
    return finish_plan(h, out);
}

int tdsolve_prepare_general(const double* lower, const double* diag, const double* upper,
                            int64_t M, int32_t P, tds_handle* out) {
    if (!out) return TDS_EINVAL;
    *out = nullptr;
    tds_plan* h = new (std::nothrow) tds_plan();
    if (!h) return TDS_ENOMEM;
    int rc = host_prepare_general(lower, diag, upper, M, P, h->host);
    if (rc) { delete h; return rc; }
    return finish_plan(h, out);
}

int tdsolve_series(tds_handle h, const void* F, void* X, int64_t N, int32_t mode, void* stream) {
    int rc = check_common(h, N, mode);
    if (rc) return rc;
    if (N == 0) return TDS_OK;
    if (!F || !X) return TDS_EINVAL;
    if (F == X && f_elem(mode) != x_elem(mode)) return TDS_EINVAL;
    const size_t cells = (size_t)h->dev.M * (size_t)N;
    if (overlap(F, cells * f_elem(mode), X, cells * x_elem(mode))) return TDS_EINVAL;
    rc = series_impl(h, F, X, N, mode, (hipStream_t)stream, mode);
    if (rc == TDS_OK) {
        void* Xv = X;
        remember(h, &F, &Xv, &N, 1, mode);
    }
    return rc;
}

int tdsolve_series_noalloc(tds_handle h, const void* F, void* X, int64_t N, int32_t mode,
                           void* stream) {
    int rc = check_common(h, N, mode);
    if (rc) return rc;
    if (N == 0) return TDS_OK;
    if (!F || !X) return TDS_EINVAL;
    if (F == X && f_elem(mode) != x_elem(mode)) return TDS_EINVAL;
    const size_t cells = (size_t)h->dev.M * (size_t)N;
    if (overlap(F, cells * f_elem(mode), X, cells * x_elem(mode))) return TDS_EINVAL;
    if (work_bytes(h, N, nullptr, nullptr, nullptr) > kNoAllocScratchBytes) return TDS_ESCRATCH;
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess) return TDS_EHIP;
    if (device != h->device) return TDS_EINVAL;
    char* base = nullptr;
    rc = noalloc_scratch(device, &base);
    if (rc) return rc;
    Work w;
    carve_work(h, N, base, w);
    return series_impl(h, F, X, N, mode, (hipStream_t)stream, mode, &w);
}

int tdsolve_components(tds_handle h, const void* F, double* Xsep, int64_t N, int32_t mode,
                       void* stream) {
    int rc = check_common(h, N, mode);
    if (rc) return rc;
    if (N == 0 || h->dev.P < 2) return TDS_OK;
    if (!F || !Xsep) return TDS_EINVAL;
    Work w;
    rc = take_work(h, N, w);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (launch_beta(h->dev, F, mode != TDS_F64, N, w.betaR, w.betaL, s) != hipSuccess)
        return TDS_EHIP;
    if (run_iface(h, w, Xsep, N, s) != hipSuccess) return TDS_EHIP;
    return TDS_OK;
}

int tdsolve_backward(tds_handle h, const void* X, const void* gX, void* gF, double* ga,
                     double* gb, int64_t N, int32_t mode, void* stream) {
    int rc = check_common(h, N, mode);
    if (rc) return rc;
    if (h->host.general) return TDS_EUNSUPPORTED;     // the adjoint solves with A^T
    if (N == 0) {
        hipStream_t s = (hipStream_t)stream;
        if (zero_f64(ga, h->dev.M - 1, s) != hipSuccess) return TDS_EHIP;
        if (zero_f64(gb, h->dev.M, s) != hipSuccess) return TDS_EHIP;
        return TDS_OK;
    }
    if (!X || !gX || !gF) return TDS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const DevTables& t = h->dev;
    if (mode == TDS_F64 || mode == TDS_F32) {
        // gX and gF have the same element type: solve straight into gF
        rc = series_impl(h, gX, gF, N, mode, s, mode);
        if (rc) return rc;
        const bool f32 = (mode == TDS_F32);
        if (launch_adjoint_reduce(t, X, gF, f32, f32, N, nullptr, ga, gb, s) != hipSuccess)
            return TDS_EHIP;
        return TDS_OK;
    }
    // X, gX are double, F (hence gF) is float: solve in FP64 into a private
    // FP64 buffer, reduce from it and round it into gF in the same pass.
    const size_t gbytes = align256(sizeof(double) * (size_t)t.M * (size_t)N);
    void* g64 = nullptr;
    hipError_t e = hipMallocAsync(&g64, gbytes, s);
    if (e == hipErrorOutOfMemory) return TDS_ENOMEM;
    if (e != hipSuccess) return TDS_EHIP;
    rc = series_impl(h, gX, g64, N, TDS_F64, s, TDS_F64);
    if (!rc && launch_adjoint_reduce(t, X, g64, false, false, N, (float*)gF, ga, gb, s) !=
                   hipSuccess)
        rc = TDS_EHIP;
    if (hipFreeAsync(g64, s) != hipSuccess && !rc) rc = TDS_EHIP;
    return rc;
}

int tdsolve_residual(tds_handle h, const void* F, const void* X, int64_t N, int32_t mode,
                     double* out, void* stream) {
    int rc = check_common(h, N, mode);
    if (rc) return rc;
    if (N == 0) return TDS_OK;
    if (!F || !X || !out) return TDS_EINVAL;
    const int64_t chunks = (h->dev.M + kReduceRowChunk - 1) / kReduceRowChunk;
    if (chunks > 65535) return TDS_EUNSUPPORTED;
    rc = ensure_work(h, sizeof(double) * 5 * (size_t)chunks * (size_t)N);
    if (rc) return rc;
    if (launch_residual(h->dev, F, X, N, mode, h->normA, (double*)general_of(h), out,
                        (hipStream_t)stream) != hipSuccess)
        return TDS_EHIP;
    return TDS_OK;
}

int tdsolve_timing_enable(tds_handle h, int32_t on) {
    if (!h) return TDS_EINVAL;
    h->timing = (on != 0);
    return TDS_OK;
}

int tdsolve_timing_read(tds_handle h, double* ms, int64_t* calls) {
    if (!h || !ms) return TDS_EINVAL;
    ms[0] = ms[1] = ms[2] = 0.0;
    const size_t ncalls = h->events_used / kTimedEvents;
    // wait for the last recorded stop event
    for (size_t c = ncalls; c-- > 0;) {
        int k = 2;
        while (k >= 0 && ((h->timed_empty[c] >> k) & 1)) --k;
        if (k < 0) continue;
        if (hipEventSynchronize(h->events[kTimedEvents * c + 2 * k + 1]) != hipSuccess)
            return TDS_EHIP;
        break;
    }
    for (size_t c = 0; c < ncalls; ++c) {
        hipEvent_t* e = h->events.data() + kTimedEvents * c;
        for (int k = 0; k < 3; ++k) {
            if ((h->timed_empty[c] >> k) & 1) continue;
            float v = 0.0f;
            if (hipEventElapsedTime(&v, e[2 * k], e[2 * k + 1]) != hipSuccess) return TDS_EHIP;
            ms[k] += v;
        }
    }
    h->timed_empty.clear();
    if (calls) *calls = (int64_t)ncalls;
    h->events_used = 0;
    return TDS_OK;
}

int tdsolve_set_interface(tds_handle h, int32_t order) {
    if (!h || h->is_batch) return TDS_EINVAL;
    if (order != TDS_IFACE_RECURRENCE && order != TDS_IFACE_DICHOTOMY &&
        order != TDS_IFACE_DENSE)
        return TDS_EINVAL;
    if (order == TDS_IFACE_DENSE && !h->dense_K && h->host.P >= 2) {
        if (h->host.P > kDenseMaxBlocks) return TDS_EUNSUPPORTED;
        std::vector<double> Kt;
        int32_t pc = 0, mr = 0;
        const int rc = dense_interface_table(h->host, Kt, &pc, &mr);
        if (rc) return rc;
        void* d = nullptr;
        const hipError_t e = hipMalloc(&d, sizeof(double) * Kt.size());
        if (e == hipErrorOutOfMemory) return TDS_ENOMEM;
        if (e != hipSuccess) return TDS_EHIP;
        if (hipMemcpy(d, Kt.data(), sizeof(double) * Kt.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
            (void)hipFree(d);
            return TDS_EHIP;
        }
        h->dense_K = (double*)d;
        h->dense_Pc = pc;
        h->dense_Mr = mr;
    }
    h->iface = order;
    return TDS_OK;
}

int tdsolve_set_fused(tds_handle h, int32_t lag, int32_t tile) {
    if (!h || h->is_batch || lag < 0 || lag > kFuseMaxLag) return TDS_EINVAL;
    if (lag > 0 && (tile < 256 || tile % 256 != 0 || tile > (1 << 20))) return TDS_EINVAL;
    h->fuse_lag = lag;
    h->fuse_cols = lag > 0 ? tile : 0;
    return TDS_OK;
}

int tdsolve_batch_set_fused(tds_handle h, int32_t lag) {
    if (!h || !h->is_batch || lag < 0 || lag > kFuseMaxLag) return TDS_EINVAL;
    h->fuse_lag = lag;
    return TDS_OK;
}

int tdsolve_set_refinement(tds_handle h, int32_t passes) {
    if (!h || passes < 0 || passes > 8) return TDS_EINVAL;
    h->passes = passes;
    return TDS_OK;
}

int tdsolve_info(tds_handle h, tds_info* info) {
    if (!h || !info || h->is_batch) return TDS_EINVAL;
    info->M = h->host.M;
    info->P = h->host.P;
    info->max_block = h->host.max_rows;
    info->dominant = h->host.dominant;
    info->refine_passes = h->passes;
    info->max_ratio = h->host.max_ratio;
    info->general = h->host.general;
    info->sweep_halves = h->has_halves ? 1 : 0;
    return TDS_OK;
}

int tdsolve_prepare_host(const double* a, const double* b, int64_t M, int32_t P, int64_t* starts,
                         double* wR, double* wL, double* rho, double* lam, double* diag_inv) {
    HostTables o;
    int rc = host_prepare(a, b, M, P, o);
    if (rc) return rc;
    if (starts) memcpy(starts, o.starts.data(), sizeof(int64_t) * (o.P + 1));
    if (wR) memcpy(wR, o.wR.data(), sizeof(double) * M);
    if (wL) memcpy(wL, o.wL.data(), sizeof(double) * M);
    if (rho) memcpy(rho, o.rho.data(), sizeof(double) * o.P);
    if (lam) memcpy(lam, o.lam.data(), sizeof(double) * o.P);
    if (diag_inv) memcpy(diag_inv, o.diag_inv.data(), sizeof(double) * M);
    return TDS_OK;
}

int tdsolve_prepare_host_general(const double* lower, const double* diag, const double* upper,
                                 int64_t M, int32_t P, int64_t* starts, double* wR, double* wL,
                                 double* rho, double* lam, double* diag_inv) {
    HostTables o;
    int rc = host_prepare_general(lower, diag, upper, M, P, o);
    if (rc) return rc;
    if (starts) memcpy(starts, o.starts.data(), sizeof(int64_t) * (o.P + 1));
    if (wR) memcpy(wR, o.wR.data(), sizeof(double) * M);
    if (wL) memcpy(wL, o.wL.data(), sizeof(double) * M);
    if (rho) memcpy(rho, o.rho.data(), sizeof(double) * o.P);
    if (lam) memcpy(lam, o.lam.data(), sizeof(double) * o.P);
    if (diag_inv) memcpy(diag_inv, o.diag_inv.data(), sizeof(double) * M);
    return TDS_OK;
}

int tdsolve_dense_table_host(const double* a, const double* b, int64_t M, int32_t P, double* K) {
    if (!K || P < 2) return TDS_EINVAL;
    if (P > kDenseMaxBlocks) return TDS_EUNSUPPORTED;
    HostTables o;
    int rc = host_prepare(a, b, M, P, o);
    if (rc) return rc;
    std::vector<double> Kt;
    int32_t pc = 0, mr = 0;
    rc = dense_interface_table(o, Kt, &pc, &mr);
    if (rc) return rc;
    // device layout Kt[kk][r] (kk = j or Pc + j) -> K[r][j] / K[r][P + j]
    const size_t w = 2 * (size_t)P;
    for (int32_t r = 0; r < P - 1; ++r)
        for (int32_t j = 0; j < P; ++j) {
            K[(size_t)r * w + j] = Kt[(size_t)j * mr + r];
            K[(size_t)r * w + P + j] = Kt[((size_t)pc + j) * mr + r];
        }
    return TDS_OK;
}

int32_t tdsolve_default_blocks(int64_t M) { return default_blocks(M); }

int tdsolve_destroy(tds_handle h) {
    if (!h) return TDS_EINVAL;
    if (h->work || h->dev_mem) (void)hipDeviceSynchronize();
    if (h->work) (void)hipFree(h->work);
    if (h->dev_mem) (void)hipFree(h->dev_mem);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    if (h->d_desc) (void)hipFree(h->d_desc);
    if (h->dense_K) {
        (void)hipDeviceSynchronize();
        (void)hipFree(h->dense_K);
    }
    delete h;
    return TDS_OK;
}

const char* tdsolve_strerror(int code) {
    switch (code) {
        case TDS_OK: return "ok";
        case TDS_EINVAL: return "invalid argument";
        case TDS_ESINGULAR: return "zero or non-finite pivot in the FP64 preliminary step";
        case TDS_ENOMEM: return "out of memory";
        case TDS_EHIP: return "HIP runtime or launch failure";
        case TDS_ENOCONV: return "refinement did not converge";
        case TDS_EUNSUPPORTED: return "unsupported size or mode";
        case TDS_ESCRATCH:
            return "work area larger than the 32 MiB fixed scratch of tdsolve_series_noalloc";
        default: return "unknown tdsolve status";
    }
}

int tdsolve_batch_prepare(int32_t K, const double* const* a, const double* const* b,
                          const int64_t* M, const int32_t* P, tds_handle* out) {
    if (!out) return TDS_EINVAL;
    *out = nullptr;
    if (K < 1 || !a || !b || !M) return TDS_EINVAL;
    tds_plan* h = new (std::nothrow) tds_plan();
    if (!h) return TDS_ENOMEM;
    h->is_batch = true;
    h->hosts.resize(K);
    h->buckets.assign(K, 0);
    bool any64 = false;
    for (int32_t k = 0; k < K; ++k) {
        int rc = host_prepare(a[k], b[k], M[k], P ? P[k] : 0, h->hosts[k]);
        if (rc) { delete h; return rc; }
        const int32_t bk = rows_bucket(h->hosts[k].max_rows);
        if (bk == 0 || bk > 64) { delete h; return TDS_EUNSUPPORTED; }   // blocks > 64 rows
        h->buckets[k] = bk;
        any64 = any64 || bk == 64;
    }
    if (hipGetDevice(&h->device) != hipSuccess) { delete h; return TDS_EHIP; }
    std::vector<unsigned char> img;
    h->devs.resize(K);
    for (int32_t k = 0; k < K; ++k) h->devs[k] = append_image(h->hosts[k], h->buckets[k], img);
    // matrices of the 64-row bucket: the sweeps with FP64 results take the
    // blocks in halves when every one of them fits them (one sweep kernel
    // per bucket)
    h->has_halves = any64;
    std::vector<HostTables> hh(K);
    for (int32_t k = 0; k < K && h->has_halves; ++k)
        if (h->buckets[k] == 64)
            h->has_halves = half_tables(h->hosts[k], kHalfRows, hh[k]) == TDS_OK;
    if (h->has_halves) {
        h->devs_h.resize(K);
        for (int32_t k = 0; k < K; ++k)
            if (h->buckets[k] == 64) h->devs_h[k] = append_image(hh[k], 0, img);
    }
    int rc = upload_image(img, &h->dev_mem);
    if (rc) { delete h; return rc; }
    for (int32_t k = 0; k < K; ++k) rebase(h->devs[k], h->dev_mem);
    for (int32_t k = 0; k < (int32_t)h->devs_h.size(); ++k)
        if (h->buckets[k] == 64) rebase(h->devs_h[k], h->dev_mem);
    *out = h;
    return TDS_OK;
}

// work items of one batch matrix in the one-launch order: beta or sweep
// items (a block x 256 right-hand sides each) and interface items (2^(lgR-1)
// right-hand sides each on a 256-thread workgroup; lgR >= 3 since G <= 64)
static int64_t fused_items(const BatchDesc& d) {
    return (int64_t)d.T.P * ((d.N + kWG - 1) / kWG);
}
static int64_t fused_scans(const BatchDesc& d) {
    const int lg = d.lgR - 1;
    return (d.N + ((int64_t)1 << lg) - 1) >> lg;
}

int tdsolve_batch_series(tds_handle h, const void* const* F, void* const* X, const int64_t* N,
                         int32_t mode, void* stream) {
    if (!h || !h->is_batch || !F || !X || !N || !valid_mode(mode)) return TDS_EINVAL;
    const int32_t K = (int32_t)h->devs.size();
    // work buffer slices and work-item ranges of every matrix; the beta and
    // sweep items of the 32-row matrices come first, then those of the
    // 64-row ones, each group numbered from 0 (one launch per group)
    std::vector<BatchDesc> desc(K);
    size_t bytes = 0;
    int64_t grp_items[2] = {0, 0}, scans = 0;
    for (int32_t k = 0; k < K; ++k) {
        const DevTables& t = h->devs[k];
        const int64_t n = N[k];
        if (n < 0 || (n > 0 && (!F[k] || !X[k]))) return TDS_EINVAL;
        if (n > 0 && F[k] == X[k] && f_elem(mode) != x_elem(mode)) return TDS_EINVAL;
        const size_t cells = (size_t)t.M * (size_t)n;
        if (n > 0 && overlap(F[k], cells * f_elem(mode), X[k], cells * x_elem(mode)))
            return TDS_EINVAL;
        BatchDesc& d = desc[k];
        d.F = F[k];
        d.X = X[k];
        d.N = n;
        d.T = t;
        const int grp = h->buckets[k] == 64 ? 1 : 0;
        d.H = (h->has_halves && grp == 1) ? h->devs_h[k] : DevTables();
        d.item0 = grp_items[grp];
        d.scan0 = scans;
        batch_scan_shape(t.P, &d.per, &d.G, &d.lgR);
        d.tile0 = 0;
        const size_t nb = align256(sizeof(double) * (size_t)t.P * (size_t)n);
        d.betaR = (double*)bytes;
        d.betaL = (double*)(bytes + nb);
        d.xsep = (double*)(bytes + 2 * nb);
        bytes += 2 * nb + align256(sizeof(double) * (size_t)(t.P > 1 ? t.P - 1 : 1) * (size_t)n);
        if (n > 0) {
            grp_items[grp] += (int64_t)t.P * ((n + kWG - 1) / kWG);
            if (t.P > 1) scans += (n + ((int64_t)1 << d.lgR) - 1) >> d.lgR;
        }
    }
    const int64_t items = grp_items[0] + grp_items[1];
    if (items == 0) {
        remember(h, F, X, N, K, mode);
        return TDS_OK;
    }
    if (items > 0x7fffffffLL || scans > 0x7fffffffLL) return TDS_EUNSUPPORTED;
    // the one-launch order (tdsolve_batch_set_fused) when every matrix with
    // work is in the 32-row bucket: its work items (per matrix the beta and
    // the sweep items, and the interface items on 256-thread workgroups),
    // written in order into the ticket table, and its counters behind the
    // work slices
    const bool fused = h->fuse_lag > 0 && grp_items[1] == 0 && K < (1 << 30);
    int64_t fitems = 0, ftiles = 0;
    size_t sync_off = 0;
    if (fused) {
        for (BatchDesc& d : desc) {
            d.tile0 = (int32_t)std::min<int64_t>(ftiles, INT32_MAX);
            if (d.N == 0) continue;
            ftiles += (d.N + kWG - 1) / kWG;
            fitems += fused_items(d);
            if (d.T.P > 1) fitems += fused_items(d) + fused_scans(d);
        }
        if (fitems > 0x7fffffffLL || ftiles > 0x7fffffffLL) return TDS_EUNSUPPORTED;
        sync_off = align256(bytes);
        bytes = sync_off + align256(sizeof(int) * (size_t)fused_batch_sync_ints(ftiles));
    }
    int rc = ensure_work(h, std::max<size_t>(bytes, 256));
    if (rc) return rc;
    for (auto& d : desc) {
        d.betaR = (double*)(general_of(h) + (size_t)d.betaR);
        d.betaL = (double*)(general_of(h) + (size_t)d.betaL);
        d.xsep = (double*)(general_of(h) + (size_t)d.xsep);
    }
    // descriptors go to the device only when they change, so that repeated
    // calls on the same buffers (e.g. replays of a captured graph) carry no
    // host-to-device copy
    // Behind the descriptors: the matrix of every beta-and-sweep item and of
    // every interface item, so that a workgroup finds its matrix by one load.
    const size_t dbytes = align256(sizeof(BatchDesc) * desc.size());
    const size_t ibytes = align256(sizeof(int32_t) * (size_t)items);
    const size_t sbytes = align256(sizeof(int32_t) * (size_t)std::max<int64_t>(scans, 1));
    const size_t total = dbytes + ibytes + sbytes + sizeof(uint64_t) * (size_t)fitems;
    const int32_t lag = fused ? h->fuse_lag : 0;
    const bool same = desc.size() == h->desc.size() && lag == h->desc_lag &&
                      memcmp(desc.data(), h->desc.data(), sizeof(BatchDesc) * desc.size()) == 0;
    if (!same) {
        std::vector<unsigned char> img;
        try {
            img.assign(total, 0);
        } catch (...) {
            return TDS_ENOMEM;
        }
        memcpy(img.data(), desc.data(), sizeof(BatchDesc) * desc.size());
        int32_t* oi = (int32_t*)(img.data() + dbytes);
        int32_t* os = (int32_t*)(img.data() + dbytes + ibytes);
        for (int32_t k = 0; k < K; ++k) {
            const BatchDesc& d = desc[k];
            if (d.N == 0) continue;
            const int64_t ni = (int64_t)d.T.P * ((d.N + kWG - 1) / kWG);
            const int64_t base = h->buckets[k] == 64 ? grp_items[0] : 0;
            for (int64_t i = 0; i < ni; ++i) oi[base + d.item0 + i] = k;
            if (d.T.P > 1) {
                const int64_t ns = (d.N + ((int64_t)1 << d.lgR) - 1) >> d.lgR;
                for (int64_t i = 0; i < ns; ++i) os[d.scan0 + i] = k;
            }
        }
        if (fused) {
            // stages: the tiles of kWG columns of every matrix, matrix by
            // matrix; stage st holds the interface items of tile st - lag,
            // the sweep items of tile st - 2 lag and the beta items of tile st
            std::vector<std::pair<int32_t, int64_t>> stage;     // (matrix, tile)
            stage.reserve((size_t)ftiles);
            for (int32_t k = 0; k < K; ++k)
                for (int64_t c = 0; c < (desc[k].N + kWG - 1) / kWG; ++c) stage.push_back({k, c});
            uint64_t* tk = (uint64_t*)(img.data() + dbytes + ibytes + sbytes);
            int64_t q = 0;
            auto put = [&](uint64_t kind, int64_t k, int64_t i) {
                tk[q++] = kind << 62 | (uint64_t)k << 32 | (uint64_t)i;
            };
            // block-major items of one tile: j tiles + c for every block j
            auto blocks = [&](uint64_t kind, int64_t st) {
                const int32_t k = stage[st].first;
                const int64_t c = stage[st].second, tiles = (desc[k].N + kWG - 1) / kWG;
                for (int64_t j = 0; j < desc[k].T.P; ++j) put(kind, k, j * tiles + c);
            };
            const int64_t S = (int64_t)stage.size();
            for (int64_t st = 0; st < S + 2 * lag; ++st) {
                const int64_t si = st - lag, ss = st - 2 * lag;
                if (si >= 0 && si < S && desc[stage[si].first].T.P > 1) {
                    // the interface items whose 2^(lgR-1) columns lie in tile si
                    const BatchDesc& d = desc[stage[si].first];
                    const int lg = d.lgR - 1;
                    const int64_t c0 = stage[si].second * kWG;
                    const int64_t c1 = std::min<int64_t>(c0 + kWG, d.N);
                    for (int64_t i = c0 >> lg; i < (c1 + ((int64_t)1 << lg) - 1) >> lg; ++i)
                        put(kFusedIface, stage[si].first, i);
                }
                if (ss >= 0 && ss < S) blocks(kFusedSweep, ss);
                if (st < S && desc[stage[st].first].T.P > 1) blocks(kFusedBeta, st);
            }
            if (q != fitems) return TDS_EHIP;     // the counts above disagree
        }
        if (h->desc_bytes < total) {
            if (h->d_desc) {
                if (hipDeviceSynchronize() != hipSuccess) return TDS_EHIP;
                (void)hipFree(h->d_desc);
                h->d_desc = nullptr;
                h->desc_bytes = 0;
            }
            if (hipMalloc(&h->d_desc, total) != hipSuccess) return TDS_ENOMEM;
            h->desc_bytes = total;
        }
        // ordered after any queued work that still reads the old descriptors
        if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return TDS_EHIP;
        if (hipMemcpy(h->d_desc, img.data(), total, hipMemcpyHostToDevice) != hipSuccess)
            return TDS_EHIP;
        h->desc = desc;
        h->desc_lag = lag;
    }
    const int32_t* own_items = (const int32_t*)((const unsigned char*)h->d_desc + dbytes);
    const int32_t* own_scans = (const int32_t*)((const unsigned char*)h->d_desc + dbytes + ibytes);
    KTime* tm = timing_slot(h);
    if (h->timing && !tm) return TDS_EHIP;
    if (fused) {
        // one launch, timed as the sweep phase
        if (tm) {
            empty_phase(h, 0);
            empty_phase(h, 1);
        }
        const uint64_t* tk =
            (const uint64_t*)((const unsigned char*)h->d_desc + dbytes + ibytes + sbytes);
        if (launch_fused_batch(h->d_desc, tk, fitems, ftiles, mode, h->passes,
                               (int*)(general_of(h) + sync_off), (hipStream_t)stream,
                               tm ? tm + 2 : nullptr) != hipSuccess)
            return TDS_EHIP;
        remember(h, F, X, N, K, mode);
        return TDS_OK;
    }
    if (tm && scans == 0) empty_phase(h, 1);
    if (launch_batch(h->d_desc, own_items, own_scans, grp_items[0], grp_items[1], scans, mode,
                     h->passes, h->has_halves, tm, (hipStream_t)stream) != hipSuccess)
        return TDS_EHIP;
    remember(h, F, X, N, K, mode);
    return TDS_OK;
}

int tdsolve_status(tds_handle h, void* stream, double* backward_err, int32_t* passes) {
    if (!h || !h->have_last) return TDS_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    const size_t K = h->last_N.size();
    // scratch of the residual kernel (partial sums, then eta and r2 per RHS)
    size_t need = 0;
    for (size_t k = 0; k < K; ++k) {
        const DevTables& t = h->is_batch ? h->devs[k] : h->dev;
        const size_t n = (size_t)h->last_N[k];
        const size_t chunks = (size_t)((t.M + kReduceRowChunk - 1) / kReduceRowChunk);
        if (n > 0 && chunks > 65535) return TDS_EUNSUPPORTED;
        need = std::max(need, 5 * chunks * n + 2 * n);
    }
    double worst = 0.0;
    bool nonfinite = false;
    if (need > 0) {
        void* buf = nullptr;
        const hipError_t e = hipMalloc(&buf, sizeof(double) * need);
        if (e == hipErrorOutOfMemory) return TDS_ENOMEM;
        if (e != hipSuccess) return TDS_EHIP;
        int rc = TDS_OK;
        std::vector<double> eta;
        for (size_t k = 0; k < K && rc == TDS_OK; ++k) {
            const int64_t n = h->last_N[k];
            if (n == 0) continue;
            const DevTables& t = h->is_batch ? h->devs[k] : h->dev;
            const size_t chunks = (size_t)((t.M + kReduceRowChunk - 1) / kReduceRowChunk);
            double* part = (double*)buf;
            double* out = part + 5 * chunks * (size_t)n;
            const double normA = h->is_batch ? norm_inf(h->hosts[k]) : h->normA;
            eta.resize((size_t)n);
            if (launch_residual(t, h->last_F[k], h->last_X[k], n, h->last_mode, normA, part, out,
                                s) != hipSuccess ||
                hipMemcpyAsync(eta.data(), out, sizeof(double) * n, hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                rc = TDS_EHIP;
                break;
            }
            for (double v : eta) {
                if (!std::isfinite(v)) nonfinite = true;
                else worst = std::max(worst, v);
            }
        }
        (void)hipFree(buf);
        if (rc) return rc;
    } else if (hipStreamSynchronize(s) != hipSuccess) {
        return TDS_EHIP;
    }
    if (backward_err) *backward_err = nonfinite ? NAN : worst;
    if (passes) *passes = h->last_passes;
    return TDS_OK;
}

}  // extern "C"

int tdsolve_strided_copy(const void* src, void* dst, int32_t f64, int64_t S, int64_t M, int64_t L,
                         const int64_t* ss, const int64_t* ds, double alpha, void* stream) {
    if (S < 0 || M < 0 || L < 0 || !ss || !ds) return TDS_EINVAL;
    if (S == 0 || M == 0 || L == 0) return TDS_OK;
    if (!src || !dst) return TDS_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (ss[k] < 0 || ds[k] < 0) return TDS_EINVAL;
    if (M > 65535) return TDS_EUNSUPPORTED;
    if (launch_strided_copy(src, dst, f64 != 0, S, M, L, ss, ds, alpha, (hipStream_t)stream) !=
        hipSuccess)
        return TDS_EHIP;
    return TDS_OK;
}
