// sbr_tsqr.hip -- panel QR of the full-to-band stage.
//
// * TSQR (Algorithm 3.2, rect-QR, on one GPU): the m x b panel is split into
//   row blocks of b rows (the last block takes the remainder, < 2b rows); each
//   block is factored by Householder QR (Lemma 3.4), then pairs of b x b R
//   factors are stacked and factored level by level up a binary tree (after
//   the first level every tree node is two stacked upper triangles).  The
//   explicit thin Q is formed top-down: the root applies its reflectors to
//   [I; 0], each node applies its reflectors to [Z; 0] with Z handed down by
//   its parent, and the leaves write their rows of Q (Q_i = W_i Z_i).
// * Householder reconstruction (Corollary 3.7): [U1, W1] = LU(Q1 - S) without
//   pivoting, S_ii = -sgn of the current pivot so |pivot| >= 1; U2 = Q2 W1^{-1}
//   (a GEMM with the explicit inverse); T = -W1 S U1^{-T}.  Then
//   (I - U T U^T)[:, :b] = Q S and (I - U T U^T)^T P = [S R; 0].
// * Ragged tail: when fewer than b rows remain below the band, the last panel
//   is reduced by unblocked Householder with the two-sided update applied one
//   reflector at a time.
//
#include <math.h>

#include "sbr_device.h"
#include "sbr_internal.h"

namespace {

struct TsqrLevelArgs {
    int b;
    int is_leaf;
    int is_root;
    // leaves
    double* P;
    int64_t ldp;
    int64_t m;
    int nleaves;
    // nodes
    double* child_slots;   // level below (b x b slots, ld b)
    int nchild;
    double* own_slots;     // this level's slots (R out for QR; Z in for apply)
    double* tau;           // this level's taus (b per node)
    // apply output for leaves
    double* Q;
    int64_t ldq;
};

struct Seg {
    double* p0;
    int64_t ld0;
    int rows0;
    double* p1;
    int64_t ld1;
    int rows1;
};

__device__ __forceinline__ Seg node_segments(const TsqrLevelArgs& a, int q) {
    Seg s;
    const int b = a.b;
    if (a.is_leaf) {
        const int64_t r0 = (int64_t)q * b;
        const int64_t rows = (q == a.nleaves - 1) ? (a.m - r0) : b;
        s.p0 = a.P + r0;
        s.ld0 = a.ldp;
        s.rows0 = (int)rows;
        s.p1 = nullptr;
        s.ld1 = 0;
        s.rows1 = 0;
    } else {
        s.p0 = a.child_slots + (int64_t)(2 * q) * b * b;
        s.ld0 = b;
        s.rows0 = b;
        if (2 * q + 1 < a.nchild) {
            s.p1 = a.child_slots + (int64_t)(2 * q + 1) * b * b;
            s.ld1 = b;
            s.rows1 = b;
        } else {
            s.p1 = nullptr;
            s.ld1 = 0;
            s.rows1 = 0;
        }
    }
    return s;
}

// Register layout of the QR / apply kernels: TPC consecutive lanes own one
// column (TPC = 8, or 2b when b < 4), lane s of the group holds the rows
// s + TPC r (r < RPT = 2b / TPC).  Column sums are DPP exchanges inside the
// group (no LDS traffic); one barrier per Householder step hands the
// reflector from its owner group to the others through LDS.
template <int B>
struct GroupQR {
    static constexpr int TPC = (2 * B < 8) ? 2 * B : 8;
    static constexpr int RPT = 2 * B / TPC;
    static constexpr int NT = B * TPC;
    static constexpr int NACC = RPT >= 4 ? 4 : RPT;   // independent partial sums
};

template <int RPT, int NACC>
__device__ __forceinline__ double dot_rows(const double* x, const double* v, int s, int tpc) {
    double acc[NACC];
#pragma unroll
    for (int a = 0; a < NACC; ++a) acc[a] = 0.0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) acc[r % NACC] += v[s + tpc * r] * x[r];
    double d = acc[0];
#pragma unroll
    for (int a = 1; a < NACC; ++a) d += acc[a];
    return d;
}

template <int B>
__global__ __launch_bounds__(GroupQR<B>::NT) void tsqr_qr_kernel(TsqrLevelArgs a) {
    typedef GroupQR<B> L;
    constexpr int TPC = L::TPC, RPT = L::RPT, NACC = L::NACC;
    __shared__ double vsh[2][2 * B];
    __shared__ double tsh[B];
    const int t = threadIdx.x, c = t / TPC, s = t % TPC;
    const int q = blockIdx.x;
    const Seg g = node_segments(a, q);
    const int rows = g.rows0 + g.rows1;
    double x[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int row = s + TPC * r;
        double v = 0.0;
        if (row < g.rows0) v = g.p0[row + (int64_t)c * g.ld0];
        else if (row < rows) v = g.p1[(row - g.rows0) + (int64_t)c * g.ld1];
        x[r] = v;
    }
    for (int k = 0; k < B; ++k) {
        double* v = vsh[k & 1];
        if (c == k) {
            double sacc[NACC];
#pragma unroll
            for (int u = 0; u < NACC; ++u) sacc[u] = 0.0;
            double xk = 0.0;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int row = s + TPC * r;
                if (row > k) sacc[r % NACC] += x[r] * x[r];
                else if (row == k) xk = x[r];
            }
            double ss = sacc[0];
#pragma unroll
            for (int u = 1; u < NACC; ++u) ss += sacc[u];
            ss = group_sum<TPC>(ss);
            xk = group_sum<TPC>(xk);
            double beta, tau, scal;
            if (ss == 0.0) {
                beta = xk; tau = 0.0; scal = 0.0;
            } else {
                const double nrm = sqrt(xk * xk + ss);
                beta = (xk >= 0.0) ? -nrm : nrm;
                tau = (beta - xk) / beta;
                scal = 1.0 / (xk - beta);
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int row = s + TPC * r;
                const double vv = (row < k) ? 0.0 : ((row == k) ? 1.0 : x[r] * scal);
                v[row] = vv;
                x[r] = (row == k) ? beta : ((row > k) ? vv : x[r]);   // selects, no branches
            }
            if (s == 0) tsh[k] = tau;
        }
        __syncthreads();
        if (c > k) {
            const double tau = tsh[k];
            if (tau != 0.0) {
                const double d = group_sum<TPC>(dot_rows<RPT, NACC>(x, v, s, TPC));
                const double f = tau * d;
#pragma unroll
                for (int r = 0; r < RPT; ++r) x[r] -= f * v[s + TPC * r];
            }
        }
    }
    // reflectors (below the diagonal) and R (on and above it) back in place
    double* R = a.own_slots + (int64_t)q * B * B;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int row = s + TPC * r;
        if (row < g.rows0) g.p0[row + (int64_t)c * g.ld0] = x[r];
        else if (row < rows) g.p1[(row - g.rows0) + (int64_t)c * g.ld1] = x[r];
        if (row < B) R[row + c * B] = (row <= c) ? x[r] : 0.0;
    }
    __syncthreads();
    if (t < B) a.tau[(int64_t)q * B + t] = tsh[t];
}

// X = H_0 ... H_{B-1} [Z; 0]: the node's explicit Q block times Z.
template <int B>
__global__ __launch_bounds__(GroupQR<B>::NT) void tsqr_apply_kernel(TsqrLevelArgs a) {
    typedef GroupQR<B> L;
    constexpr int TPC = L::TPC, RPT = L::RPT, NACC = L::NACC;
    __shared__ double vsh[2][2 * B];
    __shared__ double tsh[B];
    const int t = threadIdx.x, c = t / TPC, s = t % TPC;
    const int q = blockIdx.x;
    const Seg g = node_segments(a, q);
    const int rows = g.rows0 + g.rows1;
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
    // reflector k, element `row`: 0 above k, 1 at k, stored value below
    auto fetchv = [&](int row, int k) -> double {
        if (row > k && row < rows)
            return (row < g.rows0) ? g.p0[row + (int64_t)k * g.ld0] : g.p1[(row - g.rows0) + (int64_t)k * g.ld1];
        return (row == k) ? 1.0 : 0.0;
    };
    double vnext = (t < 2 * B) ? fetchv(t, B - 1) : 0.0;
    for (int k = B - 1; k >= 0; --k) {
        double* v = vsh[k & 1];
        if (t < 2 * B) v[t] = vnext;
        __syncthreads();
        if (k > 0 && t < 2 * B) vnext = fetchv(t, k - 1);
        const double tau = tsh[k];
        if (tau != 0.0) {
            const double d = group_sum<TPC>(dot_rows<RPT, NACC>(x, v, s, TPC));
            const double f = tau * d;
#pragma unroll
            for (int r = 0; r < RPT; ++r) x[r] -= f * v[s + TPC * r];
        }
    }
    __syncthreads();   // every read of the reflectors is done before they are overwritten
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int row = s + TPC * r;
        if (a.is_leaf) {
            if (row < g.rows0) a.Q[(int64_t)q * B + row + (int64_t)c * a.ldq] = x[r];
        } else {
            if (row < g.rows0) g.p0[row + (int64_t)c * g.ld0] = x[r];
            else if (row < rows) g.p1[(row - g.rows0) + (int64_t)c * g.ld1] = x[r];
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
void launch_level(bool qr, const TsqrLevelArgs& a, int blocks, hipStream_t s) {
    constexpr int NT = GroupQR<B>::NT;
    if (qr) tsqr_qr_kernel<B><<<blocks, NT, 0, s>>>(a);
    else tsqr_apply_kernel<B><<<blocks, NT, 0, s>>>(a);
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

}  // namespace

namespace sbr {

bool tsqr_supported(int b) {
    return b == 2 || b == 4 || b == 8 || b == 16 || b == 32 || b == 64 || b == 128;
}

int64_t tsqr_workspace_doubles(int64_t m, int b) {
    int64_t count = m / b;
    if (count < 1) count = 1;
    int64_t tot = 0;
    while (true) {
        tot += count * ((int64_t)b * b + b);
        if (count == 1) break;
        count = (count + 1) / 2;
    }
    return tot;
}

void tsqr_plan(TsqrTree& tr, int64_t m, int b, double* ws) {
    tr.b = b;
    tr.m = m;
    int64_t count = m / b;
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
        count = (count + 1) / 2;
    }
    tr.levels = lv;
}

const double* tsqr_root_r(const TsqrTree& tr) { return tr.slots[tr.levels - 1]; }

void launch_tsqr(const TsqrTree& tr, double* P, int64_t ldp, double* Q, int64_t ldq, hipStream_t s) {
    const int b = tr.b;
    TsqrLevelArgs a{};
    a.b = b;
    a.P = P;
    a.ldp = ldp;
    a.m = tr.m;
    a.nleaves = tr.count[0];
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
    return e == hipSuccess ? 0 : (int)e;
}

void launch_reconstruct(int b, const double* Q, int64_t ldq, double* U, int64_t ldu, double* T, int64_t ldt,
                        double* W1inv, double* S, hipStream_t s) {
    const size_t shm = (size_t)b * (b + 1) * sizeof(double);
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
