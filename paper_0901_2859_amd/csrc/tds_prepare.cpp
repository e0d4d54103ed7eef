// FP64 preliminary step of the parallel sweep method, on the host.
//
// Algorithm 3, step 1 asks for the rows G_k of A^{-1} at the interface rows
// (Lemma 2, eq. green_v) and the vectors Z^R_k, Z^L_k (eq. z_vector).
//
// Rows G_k: as in the paper, each is the solution of A G_k = e_k by a sweep
// (one shared forward factorization, then one elimination of e_k and one
// back substitution per interface row, O(M) each); only the two segments
// next to k are kept, since eq. beta_symn uses G_k on those alone.
//
// Vectors Z: homogeneous solutions normalised to 1 at k.  Their successive
// ratios do not depend on k and follow two first-order recurrences:
//   Z^L: l_i = z_{i-1} / z_i,  l_1 = -a_0 / b_0,
//        l_{i+1} = -a_i / (b_i + a_{i-1} l_i);
//   Z^R: r_i = z_{i+1} / z_i,  r_{M-2} = -a_{M-2} / b_{M-1},
//        r_{i-1} = -a_{i-1} / (b_i + a_i r_i),
// so Z^L_k(i) = prod_{m=i+1..k} l_m and Z^R_k(i) = prod_{m=k..i-1} r_m
// (these are the sweep coefficients alpha of the proof of Theorem 4;
// |l|, |r| <= 1 under diagonal dominance).  Theorem 2 only needs Z between
// neighbouring interface rows s_k < s_{k+1}:
//   rho_k = Z^R_{s_k}(s_{k+1}),  lam_k = Z^L_{s_{k+1}}(s_k).
// The diagonal of A^{-1} reported for checks is 1 / (b_k + a_{k-1} l_k +
// a_k r_k) away from the interface rows.
// The block sweeps (Lemma 1) use the elimination factors of each block's
// interior rows, restarted at the first interior row of every block.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "tdsolve.h"
#include "tds_internal.h"

namespace tds {

static bool bad(double v) { return !(v == v) || isinf(v); }

int32_t default_blocks(int64_t M) {
    // 64 rows per block keeps the register-resident sweep at its best size;
    // short systems use as many blocks of at least 2 rows as fit.
    if (M < 4) return 1;
    int64_t P = (M + 63) / 64;
    P = std::max<int64_t>(1, std::min<int64_t>(P, M / 2));
    return (int32_t)std::min<int64_t>(P, 1 << 20);
}

// Block-restarted elimination of every block's interior rows and the
// block's responses u, v to its left / right interface value (Lemma 1), for
// the matrix with sub-diagonal lo (A[i+1][i] = lo[i]), diagonal o.b64 and
// super-diagonal up (A[i][i+1] = up[i]).  The recurrences run in the host's
// extended precision (long double) and the tables are rounded to FP64 once:
// on a nearly singular A (the Poisson matrix) the sweeps multiply the
// boundary values, which are much larger than the right-hand side, by u and
// v, so the tables' own rounding shows directly in the residual.
using wide = long double;

// one block's elimination factors and responses; cp, rd, u, v: i1 - i0 + 1
// entries each (false: a zero or non-finite pivot)
static bool block_responses(const double* lo, const double* b, const double* up, int64_t i0,
                            int64_t i1, double cl, double cr, wide* cp, wide* rd, wide* u,
                            wide* v) {
    const int64_t n = i1 - i0 + 1;
    wide cprev = 0.0L;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t i = i0 + k;
        const wide den = (wide)b[i] - (k > 0 ? (wide)lo[i - 1] * cprev : 0.0L);
        if (den == 0.0L || bad((double)den)) return false;
        rd[k] = 1.0L / den;
        cp[k] = (k < n - 1) ? (wide)up[i] / den : 0.0L;
        cprev = cp[k];
    }
    // u = T^{-1}(-cl e_first): forward elimination then back substitution
    wide d = -(wide)cl * rd[0];
    u[0] = d;
    for (int64_t k = 1; k < n; ++k) {
        d = (0.0L - (wide)lo[i0 + k - 1] * d) * rd[k];
        u[k] = d;
    }
    for (int64_t k = n - 2; k >= 0; --k) u[k] -= cp[k] * u[k + 1];
    // v = T^{-1}(-cr e_last): only the last row is non-zero after the
    // forward elimination
    v[n - 1] = -(wide)cr * rd[n - 1];
    for (int64_t k = n - 2; k >= 0; --k) v[k] = -cp[k] * v[k + 1];
    return true;
}

static int block_tables(HostTables& o, const double* lo, const double* up) {
    const int64_t M = o.M;
    const int32_t P = o.P;
    const double* b = o.b64.data();
    const auto& s = o.starts;
    o.cp64.assign(M, 0.0);
    o.rd64.assign(M, 0.0);
    o.u.assign(M, 0.0);
    o.v.assign(M, 0.0);
    std::vector<wide> cp, rd, u, v;
    for (int32_t j = 0; j < P; ++j) {
        const int64_t i0 = (j == 0) ? s[0] : s[j] + 1;
        const int64_t i1 = s[j + 1] - 1;
        const int64_t n = i1 - i0 + 1;
        cp.resize(n);
        rd.resize(n);
        u.resize(n);
        v.resize(n);
        const double cl = (j > 0) ? lo[i0 - 1] : 0.0;     // A[i0][i0-1]
        const double cr = (j < P - 1) ? up[i1] : 0.0;     // A[i1][i1+1]
        if (!block_responses(lo, b, up, i0, i1, cl, cr, cp.data(), rd.data(), u.data(), v.data()))
            return TDS_ESINGULAR;
        for (int64_t k = 0; k < n; ++k) {
            o.cp64[i0 + k] = (double)cp[k];
            o.rd64[i0 + k] = (double)rd[k];
            o.u[i0 + k] = (double)u[k];
            o.v[i0 + k] = (double)v[k];
        }
    }
    return TDS_OK;
}

int host_prepare(const double* a, const double* b, int64_t M, int32_t P,
                 HostTables& o) {
    if (M < 1 || b == nullptr || (M > 1 && a == nullptr)) return TDS_EINVAL;
    if (M > (int64_t(1) << 40)) return TDS_EINVAL;
    if (P == 0) P = default_blocks(M);
    if (P < 1) return TDS_EINVAL;
    if (P > 1 && (int64_t)P * 2 > M) return TDS_EINVAL;
    for (int64_t i = 0; i < M; ++i)
        if (bad(b[i])) return TDS_EINVAL;
    for (int64_t i = 0; i + 1 < M; ++i)
        if (bad(a[i])) return TDS_EINVAL;

    o.M = M;
    o.P = P;
    o.starts.assign(P + 1, 0);
    const int64_t base = M / P, extra = M % P;
    o.max_rows = 0;
    for (int32_t j = 0; j < P; ++j) {
        int64_t tj = base + (j < extra ? 1 : 0);
        o.starts[j + 1] = o.starts[j] + tj;
        o.max_rows = (int32_t)std::max<int64_t>(o.max_rows, tj);
    }

    o.a64.assign(M, 0.0);
    o.b64.assign(b, b + M);
    for (int64_t i = 0; i + 1 < M; ++i) o.a64[i] = a[i];
    const double* A = o.a64.data();

    // ratio recurrences
    std::vector<double> l(M, 0.0), r(M, 0.0);
    double max_ratio = 0.0;
    for (int64_t i = 1; i < M; ++i) {
        double den = b[i - 1] + (i >= 2 ? A[i - 2] * l[i - 1] : 0.0);
        if (den == 0.0 || bad(den)) return TDS_ESINGULAR;
        l[i] = -A[i - 1] / den;
        max_ratio = std::max(max_ratio, fabs(l[i]));
    }
    for (int64_t i = M - 2; i >= 0; --i) {
        double den = b[i + 1] + (i + 2 <= M - 1 ? A[i + 1] * r[i + 1] : 0.0);
        if (den == 0.0 || bad(den)) return TDS_ESINGULAR;
        r[i] = -A[i] / den;
        max_ratio = std::max(max_ratio, fabs(r[i]));
    }
    o.max_ratio = max_ratio;

    o.diag_inv.assign(M, 0.0);
    for (int64_t k = 0; k < M; ++k) {
        double den = b[k] + (k > 0 ? A[k - 1] * l[k] : 0.0) + (k + 1 < M ? A[k] * r[k] : 0.0);
        if (den == 0.0 || bad(den)) return TDS_ESINGULAR;
        o.diag_inv[k] = 1.0 / den;
    }

    // Theorem 4's dominance condition (reported, not required)
    bool dom = true, strict = false;
    for (int64_t i = 0; i < M; ++i) {
        double off = (i > 0 ? fabs(A[i - 1]) : 0.0) + (i + 1 < M ? fabs(A[i]) : 0.0);
        if (fabs(b[i]) < off) dom = false;
        if (fabs(b[i]) > off) strict = true;
    }
    o.dominant = (dom && strict) ? 1 : 0;

    // weights of eq. beta_symn: the rows G_k of A^{-1} at the interface
    // rows k = s_1..s_{P-1} over the two segments that touch k.  As in the
    // paper's preliminary step, each G_k is the solution of A G_k = e_k by a
    // sweep.  (The closed form g_k = 1/(b_k + a_{k-1} l_k + a_k r_k) loses
    // digits to cancellation when A is close to singular -- about 1e-11
    // relative for the 4096-row Poisson matrix -- and the interface values,
    // sums of terms much larger than the solution, amplify that error.)
    o.wR.assign(M, 0.0);
    o.wL.assign(M, 0.0);
    const auto& s = o.starts;
    const bool by_sweep = (double)M * (double)(P - 1) <= 4.0e9;
    std::vector<double> piv(M), cpg(M), dg(M), xg(M);
    for (int64_t i = 0; i < M; ++i) {           // one forward factorization for all k
        piv[i] = b[i] - (i > 0 ? A[i - 1] * cpg[i - 1] : 0.0);
        if (piv[i] == 0.0 || bad(piv[i])) return TDS_ESINGULAR;
        cpg[i] = (i + 1 < M) ? A[i] / piv[i] : 0.0;
    }
    for (int32_t j = 1; j < P; ++j) {
        const int64_t k = s[j];
        const int64_t lo = s[j - 1], hi = s[j + 1];   // rows of segments j-1 and j
        if (by_sweep) {
            // forward elimination of e_k: zero above k
            dg[k] = 1.0 / piv[k];
            for (int64_t i = k + 1; i < M; ++i) dg[i] = -A[i - 1] * dg[i - 1] / piv[i];
            double x = dg[M - 1];
            xg[M - 1] = x;
            for (int64_t i = M - 2; i >= lo; --i) {
                x = (i >= k ? dg[i] : 0.0) - cpg[i] * x;
                xg[i] = x;
            }
        } else {
            xg[k] = o.diag_inv[k];
            for (int64_t i = k - 1; i >= lo; --i) xg[i] = xg[i + 1] * l[i + 1];
            for (int64_t i = k + 1; i < hi; ++i) xg[i] = xg[i - 1] * r[i - 1];
        }
        if (bad(xg[k])) return TDS_ESINGULAR;
        o.diag_inv[k] = xg[k];
        for (int64_t i = lo; i < k; ++i) o.wR[i] = xg[i];      // segment j-1, right row k
        for (int64_t i = k; i < hi; ++i) o.wL[i] = xg[i];      // segment j, left row k
    }

    // transfer factors between neighbouring interface rows
    o.rho.assign(P, 0.0);
    o.lam.assign(P, 0.0);
    for (int32_t k = 1; k + 1 <= P - 1; ++k) {
        double pr = 1.0, pl = 1.0;
        for (int64_t m = s[k]; m < s[k + 1]; ++m) pr *= r[m];
        for (int64_t m = s[k] + 1; m <= s[k + 1]; ++m) pl *= l[m];
        o.rho[k] = pr;
        o.lam[k] = pl;
    }

    o.l64 = o.a64;
    o.general = 0;
    return block_tables(o, A, A);
}

// Non-symmetric tridiagonal A (section "Nonsymmetrical matrices"): when
// lo[i] * up[i] > 0 for every i, the diagonal similarity S = D^{-1} A D with
// d_{i+1} / d_i = q_i = sqrt(lo[i] / up[i]) is symmetric, with off-diagonal
// sigma_i = sign(up[i]) sqrt(lo[i] up[i]).  The preliminary step runs on S;
// since A^{-1} = D S^{-1} D^{-1}, the rows of A^{-1} at the interface rows
// and the transfer factors follow by the ratios d_k / d_i, which are
// products of the q_m between the two rows (never the absolute d_i, which
// can overflow on long systems).  The block sweeps run on A itself.
int host_prepare_general(const double* lo, const double* diag, const double* up, int64_t M,
                         int32_t P, HostTables& o) {
    if (M < 1 || diag == nullptr || (M > 1 && (lo == nullptr || up == nullptr)))
        return TDS_EINVAL;
    std::vector<double> sig(M > 1 ? M - 1 : 1, 0.0), q(M > 1 ? M - 1 : 1, 1.0);
    for (int64_t i = 0; i + 1 < M; ++i) {
        if (bad(lo[i]) || bad(up[i])) return TDS_EINVAL;
        if (!((lo[i] > 0.0 && up[i] > 0.0) || (lo[i] < 0.0 && up[i] < 0.0)))
            return TDS_EUNSUPPORTED;
        const double sl = sqrt(fabs(lo[i])), su = sqrt(fabs(up[i]));
        sig[i] = (up[i] > 0.0 ? 1.0 : -1.0) * sl * su;
        q[i] = sl / su;
    }
    int rc = host_prepare(sig.data(), diag, M, P, o);
    if (rc) return rc;
    P = o.P;
    const auto& s = o.starts;
    // weights: wR on segment j is row s_{j+1} of A^{-1}, wL row s_j
    for (int32_t j = 0; j < P; ++j) {
        if (j < P - 1) {
            double r = 1.0;                      // d_{s_{j+1}} / d_i
            for (int64_t i = s[j + 1] - 1; i >= s[j]; --i) {
                r *= q[i];
                o.wR[i] *= r;
            }
        }
        if (j > 0) {
            double r = 1.0;                      // d_{s_j} / d_i
            for (int64_t i = s[j]; i < s[j + 1]; ++i) {
                o.wL[i] *= r;
                if (i + 1 < M) r /= q[i];
            }
        }
    }
    // transfer factors between interface rows s_k and s_{k+1}
    for (int32_t k = 1; k + 1 <= P - 1; ++k) {
        double r = 1.0;                          // d_{s_{k+1}} / d_{s_k}
        for (int64_t m = s[k]; m < s[k + 1]; ++m) r *= q[m];
        o.rho[k] *= r;
        o.lam[k] /= r;
    }
    // sweep tables of A itself
    o.a64.assign(M, 0.0);
    o.l64.assign(M, 0.0);
    for (int64_t i = 0; i + 1 < M; ++i) {
        o.a64[i] = up[i];
        o.l64[i] = lo[i];
    }
    o.general = 1;
    return block_tables(o, o.l64.data(), o.a64.data());
}

// Half-block partition for the refined sweep.  Block j's interior rows
// i0..i1 become the left half i0..m-1 (`lead` rows), the middle row
// m = i0 + lead and the right half m+1..i1; as segments of a partition of
// 2P blocks, the left half's interface row is s_j and the right half's is m,
// so block_tables gives each half its zero-boundary elimination and its
// responses u, v to the values at its two ends (Lemma 1 per half).  With x
// at the middle row written through the halves,
//     x_{m-1} = x0_{m-1} + x(s_j) u_{m-1} + x_m v_{m-1},
//     x_{m+1} = x0_{m+1} + x_m u_{m+1} + x(s_{j+1}) v_{m+1},
// row m's equation A[m][m-1] x_{m-1} + b_m x_m + A[m][m+1] x_{m+1} = f_m
// gives x_m with the factor 1 / (b_m + A[m][m-1] v_{m-1} + A[m][m+1] u_{m+1}),
// kept in mid_inv[2j+1].
int half_tables(const HostTables& o, int32_t lead, HostTables& h) {
    const int64_t M = o.M;
    const int32_t P = o.P;
    if (lead < 1 || (int64_t)P * 2 > (int64_t)1 << 30) return TDS_EUNSUPPORTED;
    h = HostTables();
    h.M = M;
    h.P = 2 * P;
    h.general = o.general;
    h.starts.assign(2 * (size_t)P + 1, 0);
    h.max_rows = 0;
    for (int32_t j = 0; j < P; ++j) {
        const int64_t i0 = (j == 0) ? o.starts[0] : o.starts[j] + 1;
        const int64_t cnt = o.starts[j + 1] - i0;
        if (cnt < lead + 2 || cnt > 2 * (int64_t)lead + 1) return TDS_EUNSUPPORTED;
        h.starts[2 * j] = o.starts[j];
        h.starts[2 * j + 1] = i0 + lead;
    }
    h.starts[2 * (size_t)P] = M;
    for (int32_t k = 0; k < h.P; ++k)
        h.max_rows = (int32_t)std::max<int64_t>(h.max_rows, h.starts[k + 1] - h.starts[k]);
    h.a64 = o.a64;
    h.l64 = o.l64;
    h.b64 = o.b64;
    h.rho.assign(h.P, 0.0);
    h.lam.assign(h.P, 0.0);
    int rc = block_tables(h, h.l64.data(), h.a64.data());
    if (rc) return rc;
    // the Schur complement b_m + A[m][m-1] v_{m-1} + A[m][m+1] u_{m+1} cancels
    // (1/16 of its terms on the Poisson matrix): it is formed from the
    // halves' extended-precision responses, not from their FP64 tables
    h.mid_inv.assign(h.P, 0.0);
    const size_t slots = 2 * (size_t)P * (size_t)lead;
    h.tw_s.assign(slots, 0.0);
    h.eR.assign(M, 0.0);
    h.tw_r.assign(slots, 1.0);
    h.tw_c.assign(slots, 0.0);
    h.tw_e.assign(slots, 0.0);
    std::vector<wide> cp, rd, u, v;
    for (int32_t j = 0; j < P; ++j) {
        const int64_t m = h.starts[2 * j + 1];
        const int64_t a0 = (j == 0) ? h.starts[0] : h.starts[2 * j] + 1;   // left half a0..m-1
        const int64_t b1 = h.starts[2 * j + 2] - 1;                          // right half m+1..b1
        const int64_t n = std::max<int64_t>(m - a0, b1 - m);
        cp.resize(n);
        rd.resize(n);
        u.resize(n);
        v.resize(n);
        const double* lo = h.l64.data();
        const double* up = h.a64.data();
        const double* bb = h.b64.data();
        if (!block_responses(lo, bb, up, a0, m - 1, j > 0 ? lo[a0 - 1] : 0.0, up[m - 1], cp.data(),
                             rd.data(), u.data(), v.data()))
            return TDS_ESINGULAR;
        const wide vA = v[m - 1 - a0];
        if (!block_responses(lo, bb, up, m + 1, b1, lo[m], j < P - 1 ? up[b1] : 0.0, cp.data(),
                             rd.data(), u.data(), v.data()))
            return TDS_ESINGULAR;
        const wide uB = u[0];
        const wide den = (wide)bb[m] + (wide)lo[m - 1] * vA + (wide)up[m] * uB;
        if (den == 0.0L || bad((double)den)) return TDS_ESINGULAR;
        h.mid_inv[2 * j + 1] = (double)(1.0L / den);
        // twisted elimination toward m, in slots k = 0..lead-1 of each half:
        // the left half top-down (slot k = row a0 + k), the right half
        // bottom-up (slot k = row m + lead - k; slots before its last row
        // b1 are padding: s = c = e = 0, r = 1).  Per slot: s, the coupling
        // to the previous slot's row; r, 1 / pivot; c, the coupling to the
        // next slot's row (the last slot's next row is m) times r; e, the
        // eliminated response to the block's outer boundary value.
        for (int hh = 0; hh < 2; ++hh) {
            const size_t base = ((size_t)2 * j + hh) * (size_t)lead;
            wide c = 0.0L, e = 0.0L;
            bool first = true;
            for (int32_t k = 0; k < lead; ++k) {
                const int64_t i = hh == 0 ? a0 + k : m + lead - k;
                if (hh == 1 && i > b1) continue;                       // padding slot
                const wide sk = first ? 0.0L : (wide)(hh == 0 ? lo[i - 1] : up[i]);
                const wide d = (wide)bb[i] - sk * c;
                if (d == 0.0L || bad((double)d)) return TDS_ESINGULAR;
                const wide r = 1.0L / d;
                const wide outer = hh == 0 ? (j > 0 ? (wide)lo[a0 - 1] : 0.0L)
                                           : (j < P - 1 ? (wide)up[b1] : 0.0L);
                e = (first ? -outer : -sk * e) * r;
                c = (wide)(hh == 0 ? up[i] : lo[i - 1]) * r;
                h.tw_s[base + k] = (double)sk;
                h.tw_r[base + k] = (double)r;
                h.tw_c[base + k] = (double)c;
                h.tw_e[base + k] = (double)e;
                first = false;
            }
        }
        // the right half's top-down elimination of a unit value at m (its
        // zero-boundary tables): e_0 = -A[m+1][m] / p_0, e_k = -A[i][i-1]
        // e_{k-1} / p_k
        {
            wide c = 0.0L, e = 0.0L;
            for (int64_t i = m + 1; i <= b1; ++i) {
                const wide d = (wide)bb[i] - (i > m + 1 ? (wide)lo[i - 1] * c : 0.0L);
                c = i < b1 ? (wide)up[i] / d : 0.0L;
                e = -(wide)lo[i - 1] * (i > m + 1 ? e : 1.0L) / d;
                h.eR[i] = (double)e;
            }
        }
    }
    return TDS_OK;
}

// Theorem 2 (eq. theor_2) written out as one coefficient matrix: for the
// interface rows k = 1..P-1,
//     x(s_k) = sum_{j<k} Z^R(s_{j+1}, s_k) beta^R_j + sum_{j>=k} Z^L(s_j, s_k) beta^L_j,
// where the ratio products between interface rows are the transfer factors
// of the preliminary step, Z^R(s_{j+1}, s_k) = rho_{j+1} ... rho_{k-1} and
// Z^L(s_j, s_k) = lam_k ... lam_{j-1} (each an empty product, 1, at j = k-1
// and j = k respectively).  Layout k-major, Kt[kk][r] with r = k-1 and
// kk = j (right part) or Pc + j (left part), Pc = P rounded up to 4, rows
// padded to Mr = (P-1) rounded up to 64; every other entry is zero.
int dense_interface_table(const HostTables& o, std::vector<double>& Kt, int32_t* Pc,
                          int32_t* Mr) {
    const int32_t P = o.P;
    if (P < 2) return TDS_EINVAL;
    const int32_t pc = (P + 3) / 4 * 4;
    const int32_t mr = (P - 1 + 63) / 64 * 64;
    const size_t kc = 2 * (size_t)pc;
    try {
        Kt.assign(kc * (size_t)mr, 0.0);
    } catch (...) {
        return TDS_ENOMEM;
    }
    for (int32_t k = 1; k <= P - 1; ++k) {
        const size_t r = (size_t)(k - 1);
        double z = 1.0;                          // Z^R(s_{j+1}, s_k), j = k-1 down to 0
        for (int32_t j = k - 1; j >= 0; --j) {
            Kt[(size_t)j * mr + r] = z;
            if (j >= 1) z *= o.rho[j];
        }
        z = 1.0;                                 // Z^L(s_j, s_k), j = k up to P-1
        for (int32_t j = k; j <= P - 1; ++j) {
            Kt[((size_t)pc + j) * mr + r] = z;
            if (j <= P - 2) z *= o.lam[j];
        }
    }
    *Pc = pc;
    *Mr = mr;
    return TDS_OK;
}

}  // namespace tds
