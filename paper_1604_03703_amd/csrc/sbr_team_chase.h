// sbr_team_chase.h -- one chase of a band halving b -> h = b/2 (Algorithm 4.2
// with k = 2) done by a team of 2h lanes of one wavefront, for small h.
//
// Lane u holds band row u of the chase's 2h-row blocks in registers: the QR
// block (rows [o, o+n_r), cols [c_q, c_q+h)), the left block (cols [o-h, o),
// j > 1), the diagonal block (rows and cols [o, o+n_r)) and the below block
// (rows [o+2h, o+2h+n_b), cols [o, o+n_r)).  Column sums are team all-reduces
// (DPP); products with T = (diag(1/tau) + strict upper part of U^T U)^{-1}
// are forward/back substitutions with G = U^T U, so T itself is never
// formed; the h x h cross-row products go through a per-team LDS block.
//   X_L -= Z (U^T X_L)            with Z = U T^T
//   X_B -= ((X_B U) T) U^T
//   W = (D U) T, V = 1/2 Z (U^T W) - W, D += U V^T + V U^T (lower part)
#pragma once
#include "sbr_device.h"

// A chase's team lies inside one wavefront (TEAM divides 64), whose lanes run
// in lock step and whose LDS accesses complete in program order, so inside a
// chase a compiler-level wavefront fence is all the synchronisation needed.
template <int TEAM>
__device__ __forceinline__ void team_sync() {
    static_assert(TEAM <= 64 && (64 % TEAM) == 0, "a team must sit inside one wavefront");
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// All-reduce sum over the TEAM lanes of an aligned team (TEAM in {2, 4, 8,
// 16}); row_mirror (lane i <-> 15 - i) joins the two 8-lane halves.
template <int TEAM>
__device__ __forceinline__ double team_sum(double v) {
    if constexpr (TEAM <= 8) {
        return group_sum<TEAM>(v);
    } else {
        v = group_sum<8>(v);
        return v + dpp_d<0x140>(v);
    }
}

// Doubles of per-team LDS scratch: U rows (2h x h), a second 2h x h block
// (the left block, then W, then V) and an h x h product.
template <int H>
constexpr int team_chase_scratch() { return 2 * (2 * H) * H + H * H; }

// One chase (i, j) at offset o (QR block columns start at cq); nr rows of the
// chase lie inside the matrix, nbr rows of the below block.  R(r, c), r >= c,
// returns a reference to band element (r, c).  Every lane of the team must
// call it (u = lane within the team).
template <int H, class Band>
__device__ __forceinline__ void team_chase(const Band& R, int o, int cq, int nr, int nbr, int j, int u,
                                           double* scr) {
    constexpr int H2 = 2 * H, TEAM = 2 * H;
    double* Us = scr;                 // U, row u at Us[u * H]
    double* Xs = scr + H2 * H;        // left block / W / V rows
    double* Ms = scr + 2 * H2 * H;    // U^T X_L, then U^T W
    const bool rv = u < nr, bvr = u < nbr;
    double q[H], d[H2], bl[H2], lf[H];
#pragma unroll
    for (int c = 0; c < H; ++c) q[c] = rv ? R(o + u, cq + c) : 0.0;
#pragma unroll
    for (int k = 0; k < H2; ++k)
        d[k] = (rv && k < nr) ? ((u >= k) ? R(o + u, o + k) : R(o + k, o + u)) : 0.0;
#pragma unroll
    for (int c = 0; c < H; ++c) lf[c] = (rv && j > 1) ? R(o + u, o - H + c) : 0.0;
#pragma unroll
    for (int k = 0; k < H2; ++k) bl[k] = (bvr && k < nr) ? R(o + H2 + u, o + k) : 0.0;

    // ---- Householder QR of the 2h x h QR block
    double tv[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const double xk = team_sum<TEAM>((u == k) ? q[k] : 0.0);
        const double ss = team_sum<TEAM>((u > k) ? q[k] * q[k] : 0.0);
        const bool none = (ss == 0.0);
        const double nrm = sqrt(xk * xk + ss);
        const double beta = none ? xk : ((xk >= 0.0) ? -nrm : nrm);
        const double tk = none ? 0.0 : (beta - xk) / beta;
        const double scal = none ? 0.0 : 1.0 / (xk - beta);
        const double v = (u == k) ? 1.0 : ((u > k) ? q[k] * scal : 0.0);
#pragma unroll
        for (int c = k + 1; c < H; ++c) {
            const double dc = team_sum<TEAM>(v * q[c]);
            q[c] -= tk * dc * v;
        }
        q[k] = (u == k) ? beta : ((u > k) ? v : q[k]);
        tv[k] = tk;
    }
    double Uu[H];
#pragma unroll
    for (int c = 0; c < H; ++c)
        Uu[c] = (tv[c] != 0.0) ? ((u == c) ? 1.0 : ((u > c) ? q[c] : 0.0)) : 0.0;
    if (rv) {
#pragma unroll
        for (int c = 0; c < H; ++c) R(o + u, cq + c) = (u <= c) ? q[c] : 0.0;
    }
    double G[H][H];
#pragma unroll
    for (int p = 0; p < H; ++p)
#pragma unroll
        for (int c = p + 1; c < H; ++c) G[p][c] = team_sum<TEAM>(Uu[p] * Uu[c]);
#pragma unroll
    for (int c = 0; c < H; ++c) Us[u * H + c] = Uu[c];
    // Z = U T^T (back substitution): Z_c = tau_c (U_c - sum_{p>c} Z_p G[c][p])
    double Z[H];
#pragma unroll
    for (int c = H - 1; c >= 0; --c) {
        double sacc = Uu[c];
#pragma unroll
        for (int p = c + 1; p < H; ++p) sacc -= Z[p] * G[c][p];
        Z[c] = tv[c] * sacc;
    }
    team_sync<TEAM>();

    // ---- below block: X_B -= ((X_B U) T) U^T
    if (nbr > 0) {
        double P[H];
#pragma unroll
        for (int c = 0; c < H; ++c) P[c] = 0.0;
#pragma unroll
        for (int k = 0; k < H2; ++k)
#pragma unroll
            for (int c = 0; c < H; ++c) P[c] += bl[k] * Us[k * H + c];
        double Wb[H];
#pragma unroll
        for (int c = 0; c < H; ++c) {
            double sacc = P[c];
#pragma unroll
            for (int p = 0; p < c; ++p) sacc -= Wb[p] * G[p][c];
            Wb[c] = tv[c] * sacc;
        }
        if (bvr) {
#pragma unroll
            for (int k = 0; k < H2; ++k) {
                double sacc = 0.0;
#pragma unroll
                for (int c = 0; c < H; ++c) sacc += Wb[c] * Us[k * H + c];
                if (k < nr) R(o + H2 + u, o + k) = bl[k] - sacc;
            }
        }
    }

    // ---- left block (j > 1): X_L -= Z (U^T X_L)
    if (j > 1) {
#pragma unroll
        for (int c = 0; c < H; ++c) Xs[u * H + c] = lf[c];
        team_sync<TEAM>();
        for (int e = u; e < H * H; e += H2) {
            const int p = e % H, c = e / H;
            double sacc = 0.0;
#pragma unroll
            for (int r = 0; r < H2; ++r) sacc += Us[r * H + p] * Xs[r * H + c];
            Ms[p * H + c] = sacc;
        }
        team_sync<TEAM>();
        if (rv) {
#pragma unroll
            for (int c = 0; c < H; ++c) {
                double sacc = 0.0;
#pragma unroll
                for (int p = 0; p < H; ++p) sacc += Z[p] * Ms[p * H + c];
                R(o + u, o - H + c) = lf[c] - sacc;
            }
        }
        team_sync<TEAM>();
    }

    // ---- diagonal block: W = (D U) T, V = 1/2 Z (U^T W) - W,
    // D += U V^T + V U^T (lower triangle)
    double W[H];
    {
        double P[H];
#pragma unroll
        for (int c = 0; c < H; ++c) P[c] = 0.0;
#pragma unroll
        for (int k = 0; k < H2; ++k)
#pragma unroll
            for (int c = 0; c < H; ++c) P[c] += d[k] * Us[k * H + c];
#pragma unroll
        for (int c = 0; c < H; ++c) {
            double sacc = P[c];
#pragma unroll
            for (int p = 0; p < c; ++p) sacc -= W[p] * G[p][c];
            W[c] = tv[c] * sacc;
        }
    }
#pragma unroll
    for (int c = 0; c < H; ++c) Xs[u * H + c] = W[c];
    team_sync<TEAM>();
    for (int e = u; e < H * H; e += H2) {
        const int p = e % H, c = e / H;
        double sacc = 0.0;
#pragma unroll
        for (int r = 0; r < H2; ++r) sacc += Us[r * H + p] * Xs[r * H + c];
        Ms[p * H + c] = sacc;
    }
    team_sync<TEAM>();
    double V[H];
#pragma unroll
    for (int c = 0; c < H; ++c) {
        double sacc = 0.0;
#pragma unroll
        for (int p = 0; p < H; ++p) sacc += Z[p] * Ms[p * H + c];
        V[c] = 0.5 * sacc - W[c];
    }
#pragma unroll
    for (int c = 0; c < H; ++c) Xs[u * H + c] = V[c];
    team_sync<TEAM>();
    if (rv) {
#pragma unroll
        for (int k = 0; k < H2; ++k) {
            if (k <= u && k < nr) {
                double sacc = 0.0;
#pragma unroll
                for (int c = 0; c < H; ++c) sacc += Uu[c] * Xs[k * H + c] + V[c] * Us[k * H + c];
                R(o + u, o + k) = d[k] + sacc;
            }
        }
    }
}
