// Internal declarations shared by the host side (prepare, C ABI) and the
// HIP kernels of the tdsolve library.  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace tds {

// Workgroup size of every per-block kernel: 4 wavefronts of 64 lanes, each
// lane one right-hand side.
constexpr int kWG = 256;
constexpr int kScanRhs = 16;      // right-hand sides per scan group (single-matrix kernel)
constexpr int kScanRhsLog2 = 4;
constexpr int kScanBatchThreads = 256;   // fused order's scan workgroup: G groups x R RHS
constexpr int kScanBatchWide = 512;      // batch scan workgroup: G groups x R RHS

// Largest block (rows of one segment) handled by the register-resident
// sweep; larger blocks take the streaming sweep, which keeps the forward
// elimination in the output array instead of registers.
constexpr int kRegMaxRows = 128;

// Device tables of one prepared matrix (all FP64 unless noted).  Row arrays
// have M entries (plus padding rows, see the upload).  `starts` has P+1
// entries (s_0 = 0 .. s_P = M).
struct DevTables {
    int64_t M = 0;
    int32_t P = 0;
    int32_t max_rows = 0;      // largest t_j
    int32_t general = 0;       // 1: non-symmetric A (sub-diagonal in l64/l32/inl*)
    int64_t* starts = nullptr;
    double* wR = nullptr;      // row of A^{-1} at the segment's right interface row
    double* wL = nullptr;      // row of A^{-1} at the segment's left interface row
    double* rho = nullptr;     // P: Z^R transfer factor from interface k to k+1
    double* lam = nullptr;     // P: Z^L transfer factor from interface k+1 to k
    double* a64 = nullptr;     // super-diagonal A[i][i+1] (0 at i = M-1)
    double* l64 = nullptr;     // sub-diagonal A[i+1][i] (= a64 for symmetric A)
    double* b64 = nullptr;     // b[i]
    double* cp64 = nullptr;    // block-restarted elimination: x_i + cp_i x_{i+1} = d_i
    double* rd64 = nullptr;    // 1 / pivot
    // Block-interior couplings, zero at every block's last interior row (so
    // a block's zero-boundary system ends there): in = super-diagonal of row
    // i (A[i][i+1]); inl = sub-diagonal, read at i-1 for row i (A[i][i-1]).
    double* in64 = nullptr;
    float* in32 = nullptr;
    double* inl64 = nullptr;
    float* inl32 = nullptr;
    // Block responses to the interface values: x = x0 + xl u + xr v, with
    // u = T^{-1}(-a_{i0-1} e_first), v = T^{-1}(-a_{i1} e_last) (Lemma 1).
    double* u = nullptr;
    double* v = nullptr;
    const double2* wpad = nullptr;         // beta weights (wR, wL) per block,
    int32_t wpad_rows = 0;                 //   padded to wpad_rows with zeros
    float* a32 = nullptr;
    float* l32 = nullptr;
    float* cp32 = nullptr;
    float* rd32 = nullptr;
    // tables of a half-block partition (half_tables): entry 2j+1 holds
    // 1 / (Schur complement of block j's middle row); P entries
    double* mid_inv = nullptr;
    // twisted elimination of a half-block partition (half_tables), in
    // slots k = 0..kHalfRows-1 of half h of block j at (2j + h) kHalfRows + k:
    // the left half's rows top-down, the right half's bottom-up (padding
    // slots first when it is shorter); s: coupling to the previous slot's
    // row, r: 1 / pivot, c: coupling to the next slot's row (m after the
    // last slot) times r, e: eliminated response to the outer boundary
    // value
    double* tw_s = nullptr;
    double* tw_r = nullptr;
    double* tw_c = nullptr;
    double* tw_e = nullptr;
    // half-block partitions, per row of a right half (zero elsewhere): its
    // zero-boundary top-down elimination of a unit value at the middle row
    // (FP32; the refined sweep's correction of x_m enters through it)
    float* eR32 = nullptr;
};

// Host-side FP64 preliminary step.  Returns a tds_status code.
struct HostTables {
    int64_t M = 0;
    int32_t P = 0;
    int32_t max_rows = 0;
    int32_t dominant = 0;
    double max_ratio = 0.0;
    std::vector<int64_t> starts;
    std::vector<double> wR, wL, rho, lam, diag_inv, a64, b64, cp64, rd64, u, v;
    std::vector<double> l64;               // sub-diagonal (a copy of a64 if symmetric)
    int32_t general = 0;                   // 1: non-symmetric A (by similarity)
    std::vector<double> mid_inv;           // half-block partitions only (half_tables)
    std::vector<double> tw_s, tw_r, tw_c, tw_e;   // half-block partitions: twisted slots
    std::vector<double> eR;                // half-block partitions: right halves' response to m
};

int host_prepare(const double* a, const double* b, int64_t M, int32_t P,
                 HostTables& out);
int host_prepare_general(const double* lo, const double* diag, const double* up,
                         int64_t M, int32_t P, HostTables& out);
int32_t default_blocks(int64_t M);
// Largest block count of the dense interface order: its table holds
// 2 P (P-1) doubles (16 MB at 1024) and its work grows as P^2 per
// right-hand side.
constexpr int32_t kDenseMaxBlocks = 1024;
// Rows of the left half when the sweeps with FP64 results split a block in
// two (k_sweep_halves): blocks of kHalfRows + 2 .. 2 kHalfRows + 1 interior
// rows.
constexpr int32_t kHalfRows = 32;
// The partition with every block of `o` split into a left half of `lead`
// interior rows, a middle row and a right half (at least one row), as
// tables for the block sweeps: 2P segments whose interface rows are the
// method's s_k and the middle rows, plus mid_inv.  TDS_EUNSUPPORTED when a
// block's length is outside lead + 2 .. 2 lead + 1 interior rows.
int half_tables(const HostTables& o, int32_t lead, HostTables& h);
// Theorem 2's coefficients as one matrix for the dense interface order
// (layout in tds_prepare.cpp); Pc, Mr: padded part width and row count.
int dense_interface_table(const HostTables& o, std::vector<double>& Kt, int32_t* Pc,
                          int32_t* Mr);

// Start and stop events of one kernel launch: with them, a launcher takes
// the kernel's own start and end timestamps (phase timing).
struct KTime {
    hipEvent_t start;
    hipEvent_t stop;
};

// Kernel launchers (tdsolve_kernels.hip).  All return hipError_t; `tm`
// (may be null) times the launch.
hipError_t launch_beta(const DevTables& t, const void* F, bool f32, int64_t N,
                       double* betaR, double* betaL, hipStream_t s,
                       const KTime* tm = nullptr);
hipError_t launch_iface(const DevTables& t, const double* betaR,
                        const double* betaL, double* xsep, int64_t N,
                        hipStream_t s, const KTime* tm = nullptr);
// the interface step by the dichotomy (Algorithm 4); SR, SL: work arrays
// of (P + 1) x N doubles
hipError_t launch_iface_dichotomy(const DevTables& t, const double* betaR,
                                  const double* betaL, double* SR, double* SL,
                                  double* xsep, int64_t N, hipStream_t s,
                                  const KTime* tm = nullptr);
// Theorem 2 as a dense product on the matrix cores (table from
// dense_interface_table)
hipError_t launch_iface_dense(const double* Kt, int32_t Pc, int32_t Mr, int32_t P,
                              const double* betaR, const double* betaL, double* xsep, int64_t N,
                              hipStream_t s, const KTime* tm = nullptr);
// `halves` (may be null): the half-block tables of t (half_tables), used by
// the sweeps with FP64 results of blocks that fit them
hipError_t launch_sweep(const DevTables& t, const void* F, void* X, int64_t N,
                        int mode, int passes, const double* xsep,
                        hipStream_t s, const KTime* tm = nullptr,
                        const DevTables* halves = nullptr);

// Fused solve (k_fused): beta weights, interface step and block sweeps in
// one launch over tiles of W right-hand sides (a multiple of 256), the
// sweeps of a tile `lag` stages (tiles) after its weights (lag >= 1).  Needs the half-block tables
// h (blocks of 33..64 rows), FP64 results, the recurrence order (Kt null) or
// the dense one (Kt, Pc, Mr as for launch_iface_dense), N even and F 8-byte
// (FP32 input) or 16-byte (FP64) aligned (fused_fits); sync: device
// ints, fused_sync_ints(N) of them, zeroed by the launcher.  `tm` times the
// fused kernel.
bool fused_fits(const DevTables& t, const DevTables* halves, const void* F, int64_t N, int mode,
                int order);
int64_t fused_sync_ints(int64_t N);
hipError_t launch_fused(const DevTables& t, const DevTables& h, const void* F, void* X,
                        int64_t N, int mode, int passes, double* betaR, double* betaL,
                        double* xsep, const double* Kt, int32_t Pc, int32_t Mr, int32_t lag,
                        int32_t W, int* sync, hipStream_t s, const KTime* tm = nullptr);

// register-sweep row bucket (32, 64, 128)// register-sweep row bucket (32, 64, 128) of a largest block size, 0 if the
// streaming sweep is needed
int32_t rows_bucket(int32_t max_rows);
// shape of the two-level interface scan: blocks per group, groups
// (<= max_groups; 16 for the batch kernels)
void scan_shape(int32_t P, int32_t max_groups, int32_t* per, int32_t* G);
// the batch kernel's shape for one matrix: per, G and log2 R with
// G R <= kScanBatchWide
void batch_scan_shape(int32_t P, int32_t* per, int32_t* G, int32_t* lgR);

// One matrix of a batch: its tables, its series and its slices of the work
// buffer, and where its work items start in the batch launches (item0: beta
// and sweep items, P * ceil(N/256) of them; scan0: interface workgroups,
// ceil(N / 2^lgR) of them, each G groups of `per` blocks x 2^lgR right-hand
// sides, from batch_scan_shape).
struct BatchDesc {
    const void* F;
    void* X;
    int64_t N;
    DevTables T;
    double* betaR;
    double* betaL;
    double* xsep;
    int64_t item0;
    int64_t scan0;
    int32_t per;
    int32_t G;
    int32_t lgR;
    int32_t tile0;     // one-launch order: the matrix's first tile of kWG columns
                       //   among the tiles of all matrices
    DevTables H;       // half-block tables (half_tables), when the batch uses them
};

// The three steps for all matrices of a batch.  The beta and sweep items of
// the matrices whose blocks fit the 32-row register bucket come first
// (items32 of them), then those of the 64-row bucket (items64; their
// BatchDesc::item0 counts from the start of that group): one launch of each
// kernel per non-empty group, one interface launch for all.  `halves`:
// every 64-row matrix's BatchDesc::H holds its half-block tables, and the
// sweeps with FP64 results take those blocks in halves.
// `tm` (may be null): start/stop events of the beta, interface and sweep
// phases, in that order (a phase of two launches starts with the first and
// stops with the second; the interface pair stays unrecorded when no
// matrix has interface rows, scans == 0).
// own_items[i] / own_scans[i]: the matrix of beta-and-sweep item i / of
// interface item i (device arrays of items32 + items64 / scans entries).
hipError_t launch_batch(const BatchDesc* D, const int32_t* own_items,
                        const int32_t* own_scans, int64_t items32, int64_t items64,
                        int64_t scans, int mode, int passes, bool halves,
                        const KTime* tm, hipStream_t s);

// The same three steps for all matrices of a batch in one launch (after a
// small one that clears `sync`), every matrix in the 32-row bucket.  tk:
// device array of `nitems` item codes in order, taken two per workgroup
// ticket (kind << 62 | matrix
// << 32 | index of the item within its matrix; kinds kFusedBeta,
// kFusedIface, kFusedSweep), the interface items on 256-thread workgroups
// (BatchDesc::lgR - 1); S: the number of tiles of kWG columns over all
// matrices (BatchDesc::tile0 numbers them).  sync: fused_batch_sync_ints(S)
// device ints.  `tm` (may be null) times the launch.
constexpr uint64_t kFusedBeta = 0, kFusedIface = 1, kFusedSweep = 2;
int64_t fused_batch_sync_ints(int64_t S);
hipError_t launch_fused_batch(const BatchDesc* D, const uint64_t* tk, int64_t nitems,
                              int64_t S, int mode, int passes, int* sync, hipStream_t s,
                              const KTime* tm);

// uniform[-1, 1) values from a counter-based generator (timing inputs)
hipError_t launch_fill_uniform(void* p, int64_t n, bool f32, uint64_t seed, hipStream_t s);
hipError_t launch_residual(const DevTables& t, const void* F, const void* X,
                           int64_t N, int mode, double normA, double* part,
                           double* out, hipStream_t s);
// gb_i, ga_i of the adjoint from X and gF; g32 (may be null): FP32 copy of
// gF written on the way
hipError_t launch_adjoint_reduce(const DevTables& t, const void* X,
                                 const void* gF, bool f32x, bool f32g,
                                 int64_t N, float* g32, double* ga,
                                 double* gb, hipStream_t s);

// dst = alpha src over S x M x L elements with the given element strides
// (tdsolve_strided_copy)
hipError_t launch_strided_copy(const void* src, void* dst, bool f64, int64_t S, int64_t M,
                               int64_t L, const int64_t* ss, const int64_t* ds, double alpha,
                               hipStream_t s);

// Rows of partial sums used by the residual and adjoint reductions.
constexpr int kReduceRowChunk = 64;

}  // namespace tds
