// sbr_tsqr.hip -- panel QR of the full-to-band stage.
//
// * TSQR (Algorithm 3.2, rect-QR, on one GPU): the m x b panel is split into
//   row blocks of 4b rows (the last block takes the remainder); each block is
//   factored by Householder QR (Lemma 3.4), then groups of up to four b x b R
//   factors are stacked and factored level by level up a 4-ary tree (a binary
//   tree for b = 128).  A wider fan-in than the binary tree of the algorithm
//   halves the number of levels, each of which is a chain of b dependent
//   Householder steps.  The explicit thin Q is formed top-down: the root
//   applies its reflectors to [I; 0], each node applies its reflectors to
//   [Z; 0] with Z handed down by its parent, and the leaves write their rows
//   of Q (Q_i = W_i Z_i).
// * Householder reconstruction (Corollary 3.7): [U1, W1] = LU(Q1 - S) without
//   pivoting, S_ii = -sgn of the current pivot so |pivot| >= 1; U2 = Q2 W1^{-1}
//   (a GEMM with the explicit inverse); T = -W1 S U1^{-T}.  Then
//   (I - U T U^T)[:, :b] = Q S and (I - U T U^T)^T P = [S R; 0].
// * Ragged tail: when fewer than b rows remain below the band, the last panel
//   is reduced by unblocked Householder with the two-sided update applied one
//   reflector at a time.
//
#include <math.h>

#include <utility>

#include "sbr_device.h"
#include "sbr_internal.h"

namespace {

// Shape of the TSQR tree for panel width B: every node stacks the R factors
// of up to F children (F B rows), every leaf is a row block of F B rows of the
// panel (the last leaf takes what is left, at least one row).  TPC consecutive
// lanes own one column; lane s of the group holds the rows s + TPC r, r < RPT.
template <int B>
struct TreeShape {
    static constexpr int F = (B >= 128) ? 2 : 4;
    static constexpr int ROWS = F * B;
    static constexpr int TPC = (ROWS < 16) ? ROWS : ((B >= 128) ? 8 : 16);
    static constexpr int RPT = ROWS / TPC;
    static constexpr int NT = B * TPC;
    static constexpr int NACC = RPT >= 4 ? 4 : RPT;   // independent partial sums
    // the apply pass keeps the node's reflectors in LDS when they fit
    static constexpr bool STAGE = (size_t)ROWS * B * sizeof(double) <= 128 * 1024;
    static constexpr bool CACHE = RPT <= 16;   // keep a reflector in registers
    // compile-time row skipping needs whole register blocks per child and is
    // kept to panels whose unrolled steps fit the register file
    static constexpr bool GENERIC = (B % TPC != 0) || B >= 128;
};

constexpr int tree_fanin(int b) { return b >= 128 ? 2 : 4; }

struct TsqrLevelArgs {
    int is_leaf;
    int is_root;
    // leaves
    double* P;
    int64_t ldp;
    int64_t m;
    // nodes
    double* child_slots;   // level below (b x b slots, ld b)
    int nchild;
    double* own_slots;     // this level's slots (R out for QR; Z in for apply)
    double* tau;           // this level's taus (b per node)
    // apply output for leaves
    double* Q;
    int64_t ldq;
};

// The stacked input of tree node (or leaf) q: rows() rows, element (row, col).
template <int B>
struct NodeView {
    double* base;
    int64_t ld;
    int rows;
    bool leaf;
    __device__ NodeView(const TsqrLevelArgs& a, int q) {
        constexpr int F = TreeShape<B>::F, ROWS = TreeShape<B>::ROWS;
        leaf = a.is_leaf != 0;
        if (leaf) {
            const int64_t r0 = (int64_t)q * ROWS;
            const int64_t left = a.m - r0;
            rows = (int)(left < ROWS ? left : ROWS);
            base = a.P + r0;
            ld = a.ldp;
        } else {
            const int nch = a.nchild - F * q;
            rows = B * (nch < F ? nch : F);
            base = a.child_slots + (int64_t)F * q * B * B;
            ld = B;
        }
    }
    // child slots are consecutive B x B blocks (ld B): row = j B + i
    __device__ __forceinline__ double* at(int row, int col) const {
        if (leaf) return base + row + (int64_t)col * ld;
        return base + (int64_t)(row / B) * B * B + (row % B) + col * B;
    }
};

// Which rows of register block r (rows s + TPC r) can be nonzero in the
// reflector of column k, for k in [TPC KR, TPC KR + TPC):
//   SKIP  none (a leaf's rows above k; in a stacked node, every row of the
//         top triangle outside its diagonal block KR and the rows of a lower
//         triangle below block KR: column k of an upper triangle is zero below
//         row k and the earlier reflectors never fill those rows);
//   MIXED some: the rows are compared with k lane by lane;
//   PLAIN all may be nonzero and all lie below row k.
// Known at compile time, so the skipped blocks cost nothing.  The generic
// shapes (panels narrower than TPC, or b = 128) use MIXED everywhere and run
// all b steps as one block.
enum RowClass { RC_SKIP, RC_MIXED, RC_PLAIN };

template <int B, bool LEAF, int KR, int R>
constexpr RowClass row_class() {
    typedef TreeShape<B> L;
    if constexpr (L::GENERIC) {
        return RC_MIXED;
    } else {
        constexpr int RB = B / L::TPC;                 // register blocks per child
        constexpr int j = LEAF ? 0 : R / RB;
        constexpr int rr = LEAF ? R : R % RB;
        if constexpr (LEAF) return rr < KR ? RC_SKIP : (rr == KR ? RC_MIXED : RC_PLAIN);
        else if constexpr (j == 0) return rr == KR ? RC_MIXED : RC_SKIP;
        else return rr > KR ? RC_SKIP : RC_PLAIN;
    }
}

template <int B>
constexpr int kr_blocks() {
    return TreeShape<B>::GENERIC ? 1 : B / TreeShape<B>::TPC;
}

template <int B>
constexpr int kr_steps() {
    return TreeShape<B>::GENERIC ? B : TreeShape<B>::TPC;
}

// Steps k = TPC KR .. of the node QR.  Step k: the group owning column k
// sums the squares below row k and publishes the unnormalised reflector
// u = x - beta e_k in LDS (its entries below k go out before the norm is
// known; the lane holding row k adds u_k = x_k - beta and beta); every later
// column applies H = I + u u^T / (beta u_k), dividing by beta u_k itself.
template <int B, bool LEAF, int KR>
__device__ __forceinline__ void qr_steps(double (&x)[TreeShape<B>::RPT], int c, int s, double* ush, double* psh,
                                         double* colsc) {
    typedef TreeShape<B> L;
    constexpr int TPC = L::TPC, RPT = L::RPT, NACC = L::NACC, ROWS = L::ROWS;
    constexpr int KN = kr_steps<B>(), K0 = KR * KN;
    for (int kk = 0; kk < KN; ++kk) {
        const int k = K0 + kk;
        double* u = ush + (k & 1) * ROWS;
        double* ps = psh + (k & 1) * 2;
        if (c == k) {
            double sacc[NACC];
#pragma unroll
            for (int w = 0; w < NACC; ++w) sacc[w] = 0.0;
            [&]<int... R>(std::integer_sequence<int, R...>) {
                ([&] {
                    constexpr RowClass rc = row_class<B, LEAF, KR, R>();
                    const int row = s + TPC * R;
                    if constexpr (rc == RC_PLAIN) {
                        sacc[R % NACC] += x[R] * x[R];
                        u[row] = x[R];
                    } else if constexpr (rc == RC_MIXED) {
                        sacc[R % NACC] += (row > k) ? x[R] * x[R] : 0.0;
                        if (row != k) u[row] = (row > k) ? x[R] : 0.0;
                    }
                }(), ...);
            }(std::make_integer_sequence<int, RPT>{});
            double ss = sacc[0];
#pragma unroll
            for (int w = 1; w < NACC; ++w) ss += sacc[w];
            ss = group_sum<TPC>(ss);
            if (s == k % TPC) {   // this lane holds row k
                double xk;
                if constexpr (L::GENERIC) {
                    xk = 0.0;
#pragma unroll
                    for (int r = 0; r < RPT; ++r) xk = (TPC * r == k - s) ? x[r] : xk;
                } else {
                    xk = x[KR];   // register block KR
                }
                double beta = xk, uk = 0.0;
                if (ss != 0.0) {
                    const double nrm = sqrt(xk * xk + ss);
                    beta = (xk >= 0.0) ? -nrm : nrm;
                    uk = xk - beta;
                }
                u[k] = uk;
                ps[0] = beta;
                ps[1] = uk;
                colsc[k] = uk;
                colsc[B + k] = beta;
                if constexpr (L::GENERIC) {
#pragma unroll
                    for (int r = 0; r < RPT; ++r) x[r] = (TPC * r == k - s) ? beta : x[r];
                } else {
                    x[KR] = beta;
                }
            }
        }
        __syncthreads();
        if (c > k) {
            const double uk = ps[1];
            if (uk != 0.0) {
                const double gk = -1.0 / (ps[0] * uk);
                double acc[NACC];
#pragma unroll
                for (int w = 0; w < NACC; ++w) acc[w] = 0.0;
                // the reflector stays in registers between the two passes
                // unless that would spill (RPT > 16: it is read twice)
                double uv[L::CACHE ? RPT : 1];
                [&]<int... R>(std::integer_sequence<int, R...>) {
                    ([&] {
                        if constexpr (row_class<B, LEAF, KR, R>() != RC_SKIP) {
                            const double ur = u[s + TPC * R];
                            if constexpr (L::CACHE) uv[R] = ur;
                            acc[R % NACC] += ur * x[R];
                        }
                    }(), ...);
                }(std::make_integer_sequence<int, RPT>{});
                double d = acc[0];
#pragma unroll
                for (int w = 1; w < NACC; ++w) d += acc[w];
                const double f = group_sum<TPC>(d) * gk;
                [&]<int... R>(std::integer_sequence<int, R...>) {
                    ([&] {
                        if constexpr (row_class<B, LEAF, KR, R>() != RC_SKIP) {
                            if constexpr (L::CACHE) x[R] -= f * uv[R];
                            else x[R] -= f * u[s + TPC * R];
                        }
                    }(), ...);
                }(std::make_integer_sequence<int, RPT>{});
            }
        }
    }
}

template <int B, bool LEAF, int KR = 0>
__device__ __forceinline__ void qr_all_steps(double (&x)[TreeShape<B>::RPT], int c, int s, double* ush, double* psh,
                                             double* colsc) {
    qr_steps<B, LEAF, KR>(x, c, s, ush, psh, colsc);
    if constexpr (KR + 1 < kr_blocks<B>()) qr_all_steps<B, LEAF, KR + 1>(x, c, s, ush, psh, colsc);
}

// Householder QR of one node or leaf (Lemma 3.4), one work-group; the
// reflectors are scaled to v = u / u_k (tau = -u_k / beta) at the end.
template <int B, bool LEAF>
__global__ __launch_bounds__(TreeShape<B>::NT) void tsqr_qr_kernel(TsqrLevelArgs a) {
    typedef TreeShape<B> L;
    constexpr int TPC = L::TPC, RPT = L::RPT, ROWS = L::ROWS;
    __shared__ double ush[2 * ROWS];
    __shared__ double psh[4];
    __shared__ double colsc[2 * B];   // u_k and beta of every column
    const int t = threadIdx.x, c = t / TPC, s = t % TPC;
    const int q = blockIdx.x;
    const NodeView<B> g(a, q);
    double x[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int row = s + TPC * r;
        x[r] = (row < g.rows) ? *g.at(row, c) : 0.0;
    }
    qr_all_steps<B, LEAF>(x, c, s, ush, psh, colsc);
    __syncthreads();
    const double my_uk = colsc[c], my_beta = colsc[B + c];
    // reflectors scaled to a unit diagonal (below it) and R (on and above it)
    // back in place
    const double rinv = (my_uk != 0.0) ? 1.0 / my_uk : 0.0;
    double* R = a.own_slots + (int64_t)q * B * B;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int row = s + TPC * r;
        const double val = (row > c) ? x[r] * rinv : x[r];
        if (row < g.rows) *g.at(row, c) = val;
        if (row < B) R[row + c * B] = (row <= c) ? val : 0.0;
    }
    if (s == 0) a.tau[(int64_t)q * B + c] = (my_uk != 0.0) ? -my_uk / my_beta : 0.0;
}

// One reflector of the apply pass: x <- (I - tau v v^T) x over the register
// blocks where reflector k can be nonzero.
template <int B, bool LEAF, int KR>
__device__ __forceinline__ void apply_reflector(double (&x)[TreeShape<B>::RPT], const double* v, double tau, int s) {
    typedef TreeShape<B> L;
    constexpr int TPC = L::TPC, RPT = L::RPT, NACC = L::NACC;
    double acc[NACC];
#pragma unroll
    for (int w = 0; w < NACC; ++w) acc[w] = 0.0;
    double vv[L::CACHE ? RPT : 1];
    [&]<int... R>(std::integer_sequence<int, R...>) {
        ([&] {
            if constexpr (row_class<B, LEAF, KR, R>() != RC_SKIP) {
                const double vr = v[s + TPC * R];
                if constexpr (L::CACHE) vv[R] = vr;
                acc[R % NACC] += vr * x[R];
            }
        }(), ...);
    }(std::make_integer_sequence<int, RPT>{});
    double d = acc[0];
#pragma unroll
    for (int w = 1; w < NACC; ++w) d += acc[w];
    const double f = tau * group_sum<TPC>(d);
    [&]<int... R>(std::integer_sequence<int, R...>) {
        ([&] {
            if constexpr (row_class<B, LEAF, KR, R>() != RC_SKIP) {
                if constexpr (L::CACHE) x[R] -= f * vv[R];
                else x[R] -= f * v[s + TPC * R];
            }
        }(), ...);
    }(std::make_integer_sequence<int, RPT>{});
}

// Reflector k, element `row`: 0 above k, 1 at k, stored value below.
template <int B>
__device__ __forceinline__ double reflector_entry(const NodeView<B>& g, int row, int k) {
    if (row > k && row < g.rows) return *g.at(row, k);
    return (row == k) ? 1.0 : 0.0;
}

template <int B, bool LEAF, int KR>
__device__ __forceinline__ void apply_steps(double (&x)[TreeShape<B>::RPT], const NodeView<B>& g, double* vst,
                                            const double* tsh, int t, int s) {
    typedef TreeShape<B> L;
    constexpr int ROWS = L::ROWS;
    constexpr int KN = kr_steps<B>(), K0 = KR * KN;
    for (int kk = KN - 1; kk >= 0; --kk) {
        const int k = K0 + kk;
        if constexpr (L::STAGE) {
            const double tau = tsh[k];
            if (tau != 0.0) apply_reflector<B, LEAF, KR>(x, vst + k * ROWS, tau, s);
        } else {
            // one reflector at a time through a double buffer
            double* v = vst + (k & 1) * ROWS;
            if (t < ROWS) v[t] = reflector_entry<B>(g, t, k);
            __syncthreads();
            const double tau = tsh[k];
            if (tau != 0.0) apply_reflector<B, LEAF, KR>(x, v, tau, s);
        }
    }
}

template <int B, bool LEAF, int KR = kr_blocks<B>() - 1>
__device__ __forceinline__ void apply_all_steps(double (&x)[TreeShape<B>::RPT], const NodeView<B>& g, double* vst,
                                                const double* tsh, int t, int s) {
    apply_steps<B, LEAF, KR>(x, g, vst, tsh, t, s);
    if constexpr (KR > 0) apply_all_steps<B, LEAF, KR - 1>(x, g, vst, tsh, t, s);
}

// X = H_0 ... H_{B-1} [Z; 0]: the node's explicit Q block times Z (the root
// starts from Z = I).  The node's reflectors are staged in LDS first when
// they fit; otherwise they pass through a two-slot LDS buffer one by one.
template <int B, bool LEAF>
__global__ __launch_bounds__(TreeShape<B>::NT) void tsqr_apply_kernel(TsqrLevelArgs a) {
    typedef TreeShape<B> L;
    constexpr int TPC = L::TPC, RPT = L::RPT, ROWS = L::ROWS, NT = L::NT;
    extern __shared__ double vst[];   // STAGE: ROWS x B reflectors; else 2 x ROWS
    __shared__ double tsh[B];
    const int t = threadIdx.x, c = t / TPC, s = t % TPC;
    const int q = blockIdx.x;
    const NodeView<B> g(a, q);
    const double* Z = a.own_slots + (int64_t)q * B * B;
    double x[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int row = s + TPC * r;
        double v = 0.0;
        if (row < B) v = a.is_root ? (row == c ? 1.0 : 0.0) : Z[row + c * B];
        x[r] = v;
    }
    if (t < B) tsh[t] = a.tau[(int64_t)q * B + t];
    if constexpr (L::STAGE) {
        // (ROWS B / NT entries a thread, the loads issued together: a loop
        // that waits for each load before the next costs that many round trips)
        static_assert((ROWS * B) % NT == 0, "staging loop");
        constexpr int PER = ROWS * B / NT;
        double ent[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = t + u * NT;
            ent[u] = reflector_entry<B>(g, idx % ROWS, idx / ROWS);
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) vst[t + u * NT] = ent[u];
    }
    __syncthreads();
    apply_all_steps<B, LEAF>(x, g, vst, tsh, t, s);
    __syncthreads();   // every read of the reflectors is done before they are overwritten
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int row = s + TPC * r;
        if (row < g.rows) {
            if (LEAF) a.Q[(int64_t)q * ROWS + row + (int64_t)c * a.ldq] = x[r];
            else *g.at(row, c) = x[r];
        }
    }
}

// Householder reconstruction for a b x b top block, one work-group.
// LDS F (b x (b+1)): Q1, then the LU factors (U1 strictly below the diagonal,
// W1 above it, the pivots of W1 kept in pv), then T (upper part, computed
// from T U1^T = -W1 S), then W1^{-1} (upper part, after W1 is reloaded).
constexpr int REC_NT = 512;

__global__ __launch_bounds__(REC_NT) void reconstruct_kernel(int b, const double* __restrict__ Q, int64_t ldq,
                                                             double* U, int64_t ldu, double* T, int64_t ldt,
                                                             double* W1inv, double* S) {
    extern __shared__ double F[];
    __shared__ double col[128];
    __shared__ double sv[128];
    __shared__ double pv[128];
    const int t = threadIdx.x;
    const int ld = b + 1;
    for (int idx = t; idx < b * b; idx += REC_NT) {
        const int i = idx % b, j = idx / b;
        F[i + j * ld] = Q[i + (int64_t)j * ldq];
    }
    __syncthreads();
    // ---- LU of Q1 - S without pivoting.  The TPR threads of a row are
    // consecutive lanes of one wave, each owning the columns = s (mod TPR).
    // Every thread derives the pivot from the unmodified diagonal entry, so
    // one barrier per step is enough.
    // threads per row: at most one wave, so a row's lanes run in lock step
    const int tpr = (REC_NT / b < 64) ? REC_NT / b : 64;
    const int row = t / tpr, sub = t % tpr;
    for (int i = 0; i < b; ++i) {
        const double aii = F[i + i * ld];
        const double si = (aii >= 0.0) ? -1.0 : 1.0;
        const double piv = aii - si;
        if (t == 0) {
            sv[i] = si;
            pv[i] = piv;
        }
        if (row > i && row < b) {
            const double l = F[row + i * ld] / piv;       // read by all lanes of the row first
            for (int c = i + 1 + ((sub - (i + 1)) % tpr + tpr) % tpr; c < b; c += tpr)
                F[row + c * ld] -= l * F[i + c * ld];
            if (sub == i % tpr) F[row + i * ld] = l;
        }
        __syncthreads();
    }
    // ---- U1 (unit lower) and W1 (upper, to T as scratch) out
    for (int idx = t; idx < b * b; idx += REC_NT) {
        const int i = idx % b, j = idx / b;
        U[i + (int64_t)j * ldu] = (i > j) ? F[i + j * ld] : (i == j ? 1.0 : 0.0);
        W1inv[i + j * b] = (i < j) ? F[i + j * ld] : (i == j ? pv[i] : 0.0);
    }
    if (t < b) S[t] = sv[t];
    __syncthreads();
    // ---- T from T U1^T = M, M = -W1 S (upper): right-looking over columns j:
    // T[:, j] = M[:, j]; M[i][j'] -= T[i][j] U1[j'][j] for i <= j < j'
    for (int idx = t; idx < b * b; idx += REC_NT) {
        const int i = idx % b, j = idx / b;
        if (i <= j) F[i + j * ld] = -((i == j) ? pv[i] : F[i + j * ld]) * sv[j];
    }
    __syncthreads();
    for (int j = 0; j + 1 < b; ++j) {
        const int w = b - 1 - j;                 // columns j+1 .. b-1
        for (int idx = t; idx < (j + 1) * w; idx += REC_NT) {
            const int i = idx % (j + 1), jp = j + 1 + idx / (j + 1);
            F[i + jp * ld] -= F[i + j * ld] * F[jp + j * ld];
        }
        __syncthreads();
    }
    for (int idx = t; idx < b * b; idx += REC_NT) {
        const int i = idx % b, j = idx / b;
        T[i + j * ldt] = (i <= j) ? F[i + j * ld] : 0.0;
    }
    __syncthreads();
    // ---- W1^{-1} (upper): reload W1 (strict upper into F, diagonal in pv),
    // then rows bottom-up: X[i][j] = R[i][j] / W1[i][i] (j >= i, R[i][i] = 1),
    // R[r][j] -= W1[r][i] X[i][j] for r < i (column i of W1 snapshotted first)
    for (int idx = t; idx < b * b; idx += REC_NT) {
        const int i = idx % b, j = idx / b;
        if (i < j) F[i + j * ld] = W1inv[i + j * b];
        else if (i == j) F[i + j * ld] = 1.0;
    }
    __syncthreads();
    for (int i = b - 1; i >= 0; --i) {
        const double inv = 1.0 / pv[i];
        for (int r = t; r < i; r += REC_NT) col[r] = F[r + i * ld];
        for (int j = i + t; j < b; j += REC_NT) F[i + j * ld] *= inv;
        __syncthreads();
        const int w = b - i;                     // columns i .. b-1
        for (int idx = t; idx < i * w; idx += REC_NT) {
            const int r = idx % i, j = i + idx / i;
            const double base = (j == i) ? 0.0 : F[r + j * ld];
            F[r + j * ld] = base - col[r] * F[i + j * ld];
        }
        __syncthreads();
    }
    for (int idx = t; idx < b * b; idx += REC_NT) {
        const int i = idx % b, j = idx / b;
        W1inv[i + j * b] = (i <= j) ? F[i + j * ld] : 0.0;
    }
}

// The same reconstruction for b = 64 with the block in registers: lane r
// holds row r (LU and T phases) or column r (the inverse of W1).  Every
// cross-lane operand is a readlane with a compile-time lane index (the loops
// are fully unrolled), so no step waits on a barrier or an LDS round trip;
// the arithmetic and its order are those of reconstruct_kernel.  Wavefront
// 0 factors; then it forms T while wavefront 1, which receives the factors
// through LDS, forms W1^{-1} (both need only the LU factors).
__device__ __forceinline__ double lane_value(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(128) void reconstruct64_kernel(const double* __restrict__ Q, int64_t ldq, double* U,
                                                            int64_t ldu, double* T, int64_t ldt, double* W1inv,
                                                            double* S) {
    constexpr int B = 64;
    __shared__ double lu[B * B];   // the LU factors, column-major (row r, column c at c B + r)
    __shared__ double pvs[B];
    const int wv = threadIdx.x >> 6, r = threadIdx.x & 63;
    double a[B];
    double sr = 0.0, pr = 0.0;             // this row's sign and pivot
    if (wv == 0) {
#pragma unroll
        for (int c = 0; c < B; ++c) a[c] = Q[r + (int64_t)c * ldq];
        // ---- LU of Q1 - S without pivoting: the pivot of step i is the
        // current diagonal entry less s_i = -sgn; rows below take the multiplier
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const double aii = lane_value(a[i], i);
            const double si = (aii >= 0.0) ? -1.0 : 1.0;
            const double piv = aii - si;
            if (r == i) {
                sr = si;
                pr = piv;
            }
            const bool below = r > i;
            const double l = a[i] / piv;
            const double lm = below ? l : 0.0;
#pragma unroll
            for (int c = i + 1; c < B; ++c) a[c] -= lm * lane_value(a[c], i);
            a[i] = below ? l : a[i];
        }
#pragma unroll
        for (int c = 0; c < B; ++c) lu[c * B + r] = a[c];
        pvs[r] = pr;
    }
    __syncthreads();
    if (wv == 0) {
        // ---- U1 (unit lower) out, S out
#pragma unroll
        for (int c = 0; c < B; ++c) U[r + (int64_t)c * ldu] = (r > c) ? a[c] : (r == c ? 1.0 : 0.0);
        S[r] = sr;
        // ---- T from T U1^T = M, M = -W1 S (upper), row r: right-looking
        // over the columns j, t[j'] -= t[j] U1[j'][j] for j' > j
        // (s_j = +-1: the products by s_j are sign flips, written as such so
        // that the only product of an update is t[j] U1[j'][j], which the
        // compiler then always fuses into the update's FMA)
        double t[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const bool pos = lane_value(sr, j) > 0.0;
            t[j] = (j > r) ? (pos ? -a[j] : a[j]) : (j == r ? (pos ? -pr : pr) : 0.0);
        }
#pragma unroll
        for (int j = 0; j + 1 < B; ++j)
#pragma unroll
            for (int jp = j + 1; jp < B; ++jp) t[jp] -= t[j] * lane_value(a[j], jp);
#pragma unroll
        for (int j = 0; j < B; ++j) T[r + (int64_t)j * ldt] = (r <= j) ? t[j] : 0.0;
    } else {
        // ---- W1^{-1} (upper), column r: bottom-up x[i] = rhs[i] / W1[i][i],
        // rhs[q] -= W1[q][i] x[i] for q < i, rhs = e_r (W1[q][i]: lane q's a[i])
#pragma unroll
        for (int c = 0; c < B; ++c) a[c] = lu[c * B + r];
        pr = pvs[r];
        const double inv_r = 1.0 / pr;
        double x[B];
#pragma unroll
        for (int i = 0; i < B; ++i) x[i] = (i == r) ? 1.0 : 0.0;
#pragma unroll
        for (int i = B - 1; i >= 0; --i) {
            x[i] *= lane_value(inv_r, i);
#pragma unroll
            for (int q = 0; q < i; ++q) x[q] -= lane_value(a[i], q) * x[i];
        }
#pragma unroll
        for (int i = 0; i < B; ++i) W1inv[i + (int64_t)r * B] = (i <= r) ? x[i] : 0.0;
    }
}

__global__ void zero_block_kernel(int64_t m, int64_t nc, double* X, int64_t ldx) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * nc) return;
    X[idx % m + (idx / m) * ldx] = 0.0;
}

__global__ void panel_writeback_kernel(int64_t m, int b, double* P, int64_t ldp, const double* __restrict__ R,
                                       const double* __restrict__ S) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * b) return;
    const int64_t i = idx % m;
    const int j = (int)(idx / m);
    double v = 0.0;
    if (i < b && i <= j) v = S[i] * R[i + (int64_t)j * b];
    P[i + j * ldp] = v;
}

// Ragged tail, one work-group: P (m x b, m < b) panel rows, A22 (m x m).
constexpr int TAIL_NT = 256;

__global__ __launch_bounds__(TAIL_NT) void f2b_tail_kernel(int m, int b, double* P, int64_t ldp, double* A,
                                                           int64_t lda) {
    __shared__ double v[128];
    __shared__ double p[128];
    __shared__ double red[TAIL_NT];
    __shared__ double sc[4];
    const int t = threadIdx.x;
    for (int k = 0; k + 1 < m; ++k) {
        // norm of P[k+1:m, k]
        double ss = 0.0;
        for (int r = k + 1 + t; r < m; r += TAIL_NT) ss += P[r + k * ldp] * P[r + k * ldp];
        red[t] = ss;
        __syncthreads();
        for (int o = TAIL_NT / 2; o > 0; o >>= 1) {
            if (t < o) red[t] += red[t + o];
            __syncthreads();
        }
        if (t == 0) {
            const double xk = P[k + k * ldp];
            const double s2 = red[0];
            double beta, tau, scal;
            if (s2 == 0.0) {
                beta = xk; tau = 0.0; scal = 0.0;
            } else {
                const double nrm = sqrt(xk * xk + s2);
                beta = (xk >= 0.0) ? -nrm : nrm;
                tau = (beta - xk) / beta;
                scal = 1.0 / (xk - beta);
            }
            sc[0] = beta; sc[1] = tau; sc[2] = scal;
        }
        __syncthreads();
        const double beta = sc[0], tau = sc[1], scal = sc[2];
        for (int r = t; r < m; r += TAIL_NT) v[r] = (r < k) ? 0.0 : (r == k ? 1.0 : P[r + k * ldp] * scal);
        __syncthreads();
        if (tau == 0.0) continue;   // uniform
        for (int r = k + t; r < m; r += TAIL_NT) P[r + k * ldp] = (r == k) ? beta : 0.0;
        // remaining panel columns: P[k:, c] -= tau v (v^T P[k:, c])
        for (int cc = k + 1 + t; cc < b; cc += TAIL_NT) {
            double dot = 0.0;
            for (int r = k; r < m; ++r) dot += v[r] * P[r + cc * ldp];
            const double f = tau * dot;
            for (int r = k; r < m; ++r) P[r + cc * ldp] -= f * v[r];
        }
        // two-sided on all of A22 (v is zero above row k): p = tau A v (lower
        // storage), w = p - (tau/2)(p^T v) v, A -= v w^T + w v^T
        for (int r = t; r < m; r += TAIL_NT) {
            double acc = 0.0;
            for (int kk = k; kk < m; ++kk) {
                const double arr = (r >= kk) ? A[r + kk * lda] : A[kk + r * lda];
                acc += arr * v[kk];
            }
            p[r] = tau * acc;
        }
        __syncthreads();
        double pv = 0.0;
        for (int r = t; r < m; r += TAIL_NT) pv += p[r] * v[r];
        red[t] = pv;
        __syncthreads();
        for (int o = TAIL_NT / 2; o > 0; o >>= 1) {
            if (t < o) red[t] += red[t + o];
            __syncthreads();
        }
        const double cfac = 0.5 * tau * red[0];
        __syncthreads();
        for (int r = t; r < m; r += TAIL_NT) p[r] -= cfac * v[r];
        __syncthreads();
        for (int idx = t; idx < m * m; idx += TAIL_NT) {
            const int r = idx % m, cc = idx / m;
            if (r >= cc) A[r + cc * lda] -= v[r] * p[cc] + p[r] * v[cc];
        }
        __syncthreads();
    }
}

template <int B>
size_t apply_lds_bytes() {
    typedef TreeShape<B> L;
    return (L::STAGE ? (size_t)L::ROWS * B : 2 * (size_t)L::ROWS) * sizeof(double);
}

template <int B>
void launch_level(bool qr, const TsqrLevelArgs& a, int blocks, hipStream_t s) {
    constexpr int NT = TreeShape<B>::NT;
    if (qr) {
        if (a.is_leaf) tsqr_qr_kernel<B, true><<<blocks, NT, 0, s>>>(a);
        else tsqr_qr_kernel<B, false><<<blocks, NT, 0, s>>>(a);
    } else {
        if (a.is_leaf) tsqr_apply_kernel<B, true><<<blocks, NT, apply_lds_bytes<B>(), s>>>(a);
        else tsqr_apply_kernel<B, false><<<blocks, NT, apply_lds_bytes<B>(), s>>>(a);
    }
}

void launch_level_b(int b, bool qr, const TsqrLevelArgs& a, int blocks, hipStream_t s) {
    switch (b) {
        case 2: launch_level<2>(qr, a, blocks, s); break;
        case 4: launch_level<4>(qr, a, blocks, s); break;
        case 8: launch_level<8>(qr, a, blocks, s); break;
        case 16: launch_level<16>(qr, a, blocks, s); break;
        case 32: launch_level<32>(qr, a, blocks, s); break;
        case 64: launch_level<64>(qr, a, blocks, s); break;
        case 128: launch_level<128>(qr, a, blocks, s); break;
        default: break;
    }
}

template <int B>
hipError_t set_apply_lds() {
    hipError_t e = hipFuncSetAttribute((const void*)tsqr_apply_kernel<B, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)apply_lds_bytes<B>());
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)tsqr_apply_kernel<B, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)apply_lds_bytes<B>());
    return e;
}

}  // namespace

namespace sbr {

bool tsqr_supported(int b) {
    return b == 2 || b == 4 || b == 8 || b == 16 || b == 32 || b == 64 || b == 128;
}

int64_t tsqr_workspace_doubles(int64_t m, int b) {
    const int F = tree_fanin(b);
    const int64_t rows = (int64_t)F * b;
    int64_t count = (m + rows - 1) / rows;
    if (count < 1) count = 1;
    int64_t tot = 0;
    while (true) {
        tot += count * ((int64_t)b * b + b);
        if (count == 1) break;
        count = (count + F - 1) / F;
    }
    return tot;
}

void tsqr_plan(TsqrTree& tr, int64_t m, int b, double* ws) {
    const int F = tree_fanin(b);
    const int64_t rows = (int64_t)F * b;
    tr.b = b;
    tr.m = m;
    int64_t count = (m + rows - 1) / rows;
    if (count < 1) count = 1;
    int lv = 0;
    double* p = ws;
    while (true) {
        tr.count[lv] = (int)count;
        tr.slots[lv] = p;
        p += count * (int64_t)b * b;
        tr.tau[lv] = p;
        p += count * (int64_t)b;
        ++lv;
        if (count == 1) break;
        count = (count + F - 1) / F;
    }
    tr.levels = lv;
}

const double* tsqr_root_r(const TsqrTree& tr) { return tr.slots[tr.levels - 1]; }

void launch_tsqr(const TsqrTree& tr, double* P, int64_t ldp, double* Q, int64_t ldq, hipStream_t s) {
    const int b = tr.b;
    TsqrLevelArgs a{};
    a.P = P;
    a.ldp = ldp;
    a.m = tr.m;
    a.Q = Q;
    a.ldq = ldq;
    // up-sweep
    for (int lv = 0; lv < tr.levels; ++lv) {
        a.is_leaf = (lv == 0);
        a.is_root = (lv == tr.levels - 1);
        a.child_slots = lv ? tr.slots[lv - 1] : nullptr;
        a.nchild = lv ? tr.count[lv - 1] : 0;
        a.own_slots = tr.slots[lv];
        a.tau = tr.tau[lv];
        launch_level_b(b, true, a, tr.count[lv], s);
    }
    // down-sweep: explicit Q
    for (int lv = tr.levels - 1; lv >= 0; --lv) {
        a.is_leaf = (lv == 0);
        a.is_root = (lv == tr.levels - 1);
        a.child_slots = lv ? tr.slots[lv - 1] : nullptr;
        a.nchild = lv ? tr.count[lv - 1] : 0;
        a.own_slots = tr.slots[lv];
        a.tau = tr.tau[lv];
        launch_level_b(b, false, a, tr.count[lv], s);
    }
}

int init_tsqr_attributes() {
    const int bytes = 128 * 129 * (int)sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void*)reconstruct_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       bytes);
    if (e == hipSuccess) e = set_apply_lds<2>();
    if (e == hipSuccess) e = set_apply_lds<4>();
    if (e == hipSuccess) e = set_apply_lds<8>();
    if (e == hipSuccess) e = set_apply_lds<16>();
    if (e == hipSuccess) e = set_apply_lds<32>();
    if (e == hipSuccess) e = set_apply_lds<64>();
    if (e == hipSuccess) e = set_apply_lds<128>();
    return e == hipSuccess ? 0 : (int)e;
}

void launch_reconstruct(int b, const double* Q, int64_t ldq, double* U, int64_t ldu, double* T, int64_t ldt,
                        double* W1inv, double* S, hipStream_t s) {
    const size_t shm = (size_t)b * (b + 1) * sizeof(double);
    if (b == 64) {
        reconstruct64_kernel<<<1, 128, 0, s>>>(Q, ldq, U, ldu, T, ldt, W1inv, S);
        return;
    }
    reconstruct_kernel<<<1, REC_NT, shm, s>>>(b, Q, ldq, U, ldu, T, ldt, W1inv, S);
}

void launch_zero_block(int64_t m, int64_t nc, double* X, int64_t ldx, hipStream_t s) {
    const int64_t tot = m * nc;
    if (tot <= 0) return;
    zero_block_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(m, nc, X, ldx);
}

void launch_panel_writeback(int64_t m, int b, double* P, int64_t ldp, const double* R, const double* S,
                            hipStream_t s) {
    const int64_t tot = m * b;
    panel_writeback_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(m, b, P, ldp, R, S);
}

void launch_f2b_tail(int64_t m, int b, double* P, int64_t ldp, double* A22, int64_t lda, hipStream_t s) {
    if (m < 2) return;
    f2b_tail_kernel<<<1, TAIL_NT, 0, s>>>((int)m, b, P, ldp, A22, lda);
}

}  // namespace sbr
