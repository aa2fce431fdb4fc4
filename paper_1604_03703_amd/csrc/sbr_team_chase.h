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
#include <utility>

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

// Chases done by one lane (h = 1) or by a small team of lanes (h = 2, 4)
// that own a whole sweep, in two phases so that consecutive sweeps can run
// two chases apart: the QR phase reads the chase's QR block, forms the
// reflectors and writes [R; 0] back; the update phase applies them to the
// left block (X_L <- Q^T X_L), the below block (X_B <- X_B Q) and the
// diagonal block (D <- Q^T D Q).  The caller puts a work-group barrier
// between the phases of one step: a neighbouring sweep's update phase reads
// entries of this chase's QR block, and this chase's update phase reads
// entries of the neighbour's.
//
// The sweep keeps the chase's below block in registers: it is the next
// chase's QR block (its first h columns) and left block (its last h
// columns).  No other sweep writes those entries in between (the neighbour
// one step behind touches the QR part only after the QR phase has stored it,
// and never the left part), so a chase loads only its diagonal and below
// blocks (and, for j = 1, its QR block).
//
// The band window is addressed through one LDS pointer per column: the ring
// holds column c at slot c mod WC (LDW doubles, diagonal offset r - c), and
// every element offset inside a column is a compile-time constant.
template <int H>
struct LaneCarry {
    double b[2 * H][2 * H];   // rows o + 2h + r, columns o + c of the last chase
};

// col[x] -> column o - 2h + x, x < 4h
template <int H, int WC, int LDW>
__device__ __forceinline__ void chase_columns(double* ring, int o, double* (&col)[4 * H]) {
    int sl = (o + WC - 2 * H) % WC;
#pragma unroll
    for (int x = 0; x < 4 * H; ++x) {
        col[x] = ring + sl * LDW;
        sl = (sl + 1 == WC) ? 0 : sl + 1;
    }
}

// h = 1: the reflection of the 2 x 1 QR block x is the symmetric 2 x 2 matrix
// [[c, s], [s, -c]] with (c, s) = (x0, x1) / beta, beta = -sgn(x0) ||x||,
// applied in closed form (the identity when x1 = 0).  Columns never reach
// past the matrix end (o <= n - 2); rows past it read and keep zeros.
struct LaneRot {
    double c, s;
};

template <int WC, int LDW>
__device__ __forceinline__ void lane_chase_qr(double* ring, int o, bool first, const LaneCarry<1>& cy,
                                              LaneRot& rot) {
    double* col[4];
    chase_columns<1, WC, LDW>(ring, o, col);
    // element (o + r, o - 2 + x) is col[x][2 + r - x]; the QR block is column
    // o - 1 (x = 1) for j = 1, else column o - 2 (x = 0), in the carry
    const double x0 = first ? col[1][1] : cy.b[0][0];
    const double x1 = first ? col[1][2] : cy.b[1][0];
    const bool none = (x1 == 0.0);
    const double rinv = rsqrt(x0 * x0 + x1 * x1);
    const double sg = (x0 >= 0.0) ? -1.0 : 1.0;          // sign of beta
    rot.c = none ? 1.0 : -fabs(x0) * rinv;
    rot.s = none ? 0.0 : sg * x1 * rinv;
    const double r0 = none ? x0 : sg * (x0 * x0 + x1 * x1) * rinv;
    double* qc = first ? col[1] + 1 : col[0] + 2;
    qc[0] = r0;
    qc[1] = 0.0;
}

template <int WC, int LDW>
__device__ __forceinline__ void lane_chase_update(double* ring, int o, bool first, LaneCarry<1>& cy,
                                                  const LaneRot& rot) {
    double* col[4];
    chase_columns<1, WC, LDW>(ring, o, col);
    const double c = rot.c, s = rot.s;
    if (!first) {
        // left block: column o - 1, rows o and o + 1
        const double l0 = cy.b[0][1], l1 = cy.b[1][1];
        col[1][1] = c * l0 + s * l1;
        col[1][2] = s * l0 - c * l1;
    }
    {
        const double da = col[2][0], db = col[2][1], dd = col[3][0];
        const double cc = c * c, ss2 = s * s, cs = c * s;
        const double t2 = 2.0 * cs * db;
        col[2][0] = cc * da + t2 + ss2 * dd;
        col[3][0] = ss2 * da - t2 + cc * dd;
        col[2][1] = cs * (da - dd) + (ss2 - cc) * db;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        // below block row o + 2 + r: columns o (x = 2) and o + 1 (x = 3)
        const double e0 = col[2][2 + r], e1 = col[3][1 + r];
        const double f0 = c * e0 + s * e1, f1 = s * e0 - c * e1;
        col[2][2 + r] = f0;
        col[3][1 + r] = f1;
        cy.b[r][0] = f0;
        cy.b[r][1] = f1;
    }
}

// Broadcast lane SRC of each aligned group of T lanes (T in {2, 4, 16}) to
// the whole group: quad_perm (lane q of a quad reads lane sel[q]) inside a
// quad, row_newbcast (every lane of a 16-lane row reads lane SRC) for a row.
template <int T, int SRC>
__device__ __forceinline__ double group_bcast(double v) {
    static_assert(T == 2 || T == 4 || T == 16, "group size");
    constexpr int CTRL = (T == 16) ? (0x150 + SRC)
                       : (T == 4) ? (SRC | (SRC << 2) | (SRC << 4) | (SRC << 6))
                                  : (SRC | (SRC << 2) | ((2 + SRC) << 4) | ((2 + SRC) << 6));
    return dpp_d<CTRL>(v);
}

// out[s'] = v of lane s' of the group, for every s' < T
template <int T>
__device__ __forceinline__ void group_gather(double v, double* out) {
    [&]<int... S>(std::integer_sequence<int, S...>) {
        ((out[S] = group_bcast<T, S>(v)), ...);
    }(std::make_integer_sequence<int, T>{});
}

// Every lane of a team of T gets the whole 2h-vector whose rows s + T i the
// lanes hold: by DPP broadcasts inside a quad, through the team's LDS slice
// (2h doubles, written then read back by the same wavefront) for T = 16,
// where 16 broadcasts per vector would keep too many registers live.
template <int H, int T>
__device__ __forceinline__ void team_gather(const double (&loc)[2 * H / T], double (&full)[2 * H], double* buf,
                                            int s) {
    constexpr int RL = 2 * H / T;
    if constexpr (T <= 4) {
#pragma unroll
        for (int i = 0; i < RL; ++i) group_gather<T>(loc[i], full + T * i);
    } else {
#pragma unroll
        for (int i = 0; i < RL; ++i) buf[s + T * i] = loc[i];
        team_sync<T>();
#pragma unroll
        for (int r = 0; r < 2 * H; ++r) full[r] = buf[r];
        team_sync<T>();
    }
}

// h = 2 and 4: a team of T lanes (T in {2, 4, 16}, T <= 2h) per sweep; lane s
// holds the rows s + T i (i < 2h / T) of every 2h-row block of the chase, and
// carries its rows of the below block into the next chase.  Reflector k is
// kept unnormalised, u = x - beta e_k, so that H_k = I + g u u^T with
// g = 1 / (beta u_k): one division per reflector and no scaling of the
// vector.  Q = H_0 ... H_{h-1} is applied one reflector at a time, each
// two-sided diagonal step being D += u w^T + w u^T with p = g D u,
// w = p + (g/2)(u^T p) u.  Column sums are team all-reduces; the reflector
// and w are gathered into every lane.
//
// GUARD: columns past the matrix end may fall inside the chase (o + 2h > n);
// otherwise every column is inside and rows past n read (and keep) zeros.
template <int H, int T>
struct TeamRefl {
    double u[H][2 * H / T];   // this lane's rows of reflector k
    double g[H];
};

template <int H, int T, int WC, int LDW, bool GUARD>
__device__ __forceinline__ void team_lane_chase_qr(double* ring, int o, bool first, int nr, int s,
                                                   const LaneCarry<H>& cy, TeamRefl<H, T>& rf) {
    constexpr int H2 = 2 * H, RL = H2 / T;
    static_assert(H2 % T == 0, "rows per lane");
    double* col[4 * H];
    chase_columns<H, WC, LDW>(ring, o, col);
    // element (o + r, o - 2h + x): diagonal offset 2h + r - x
    auto at = [&](int r, int x) -> double& { return col[x][H2 + r - x]; };
    // the QR block: columns o - h .. (x = h ..) for j = 1, else the carry
    double q[RL][H];
#pragma unroll
    for (int i = 0; i < RL; ++i) {
        const int r = s + T * i;
#pragma unroll
        for (int c = 0; c < H; ++c) {
            double m = at(r, H + c);
            if (GUARD) m = (r < nr) ? m : 0.0;
            q[i][c] = first ? m : cy.b[i][c];
        }
    }
#pragma unroll
    for (int k = 0; k < H; ++k) {
        // x_k sits in lane k % T, row slot k / T
        double ssp = 0.0, xkp = 0.0;
#pragma unroll
        for (int i = 0; i < RL; ++i) {
            const int r = s + T * i;
            ssp += (r > k) ? q[i][k] * q[i][k] : 0.0;
            xkp = (r == k) ? q[i][k] : xkp;
        }
        const double ss = group_sum<T>(ssp);
        const double xk = group_sum<T>(xkp);
        const bool none = (ss == 0.0);
        const double nrm = sqrt(xk * xk + ss);
        const double beta = none ? xk : ((xk >= 0.0) ? -nrm : nrm);
        const double uk = xk - beta;
        const double g = none ? 0.0 : 1.0 / (beta * uk);
#pragma unroll
        for (int i = 0; i < RL; ++i) {
            const int r = s + T * i;
            rf.u[k][i] = (r < k) ? 0.0 : ((r == k) ? uk : q[i][k]);
            q[i][k] = (r == k) ? beta : ((r > k) ? 0.0 : q[i][k]);
        }
        rf.g[k] = g;
        // the QR block's columns c > k: X += g u (u^T X)
#pragma unroll
        for (int c = k + 1; c < H; ++c) {
            double p = 0.0;
#pragma unroll
            for (int i = 0; i < RL; ++i) p += rf.u[k][i] * q[i][c];
            const double f = g * group_sum<T>(p);
#pragma unroll
            for (int i = 0; i < RL; ++i) q[i][c] += f * rf.u[k][i];
        }
    }
#pragma unroll
    for (int i = 0; i < RL; ++i) {
        const int r = s + T * i;
        if (!GUARD || r < nr) {
#pragma unroll
            for (int c = 0; c < H; ++c) at(r, first ? H + c : c) = q[i][c];
        }
    }
}

template <int H, int T, int WC, int LDW, bool GUARD>
__device__ __forceinline__ void team_lane_chase_update(double* ring, int o, bool first, int nr, int nbr, int s,
                                                       LaneCarry<H>& cy, const TeamRefl<H, T>& rf,
                                                       double* tbuf) {
    constexpr int H2 = 2 * H, RL = H2 / T;
    double* col[4 * H];
    chase_columns<H, WC, LDW>(ring, o, col);
    auto at = [&](int r, int x) -> double& { return col[x][H2 + r - x]; };
    // the left block (columns o - h .., j > 1) from the carry, this lane's
    // full rows of the diagonal block and its rows of the below block
    double lf[RL][H], d[RL][H2], bl[RL][H2];
#pragma unroll
    for (int i = 0; i < RL; ++i) {
        const int r = s + T * i;
#pragma unroll
        for (int c = 0; c < H; ++c) lf[i][c] = cy.b[i][H + c];
        // D[r][c] = band(o + max, o + min); column o + r (a lane-dependent
        // column) through its own pointer
        const double* colr = ring + ((o + r) % WC) * LDW;
#pragma unroll
        for (int c = 0; c < H2; ++c) {
            const double* pa = (c <= r) ? col[H2 + c] + (r - c) : colr + (c - r);
            double v = *pa;
            if (GUARD) v = (r < nr && c < nr) ? v : 0.0;
            d[i][c] = v;
        }
#pragma unroll
        for (int c = 0; c < H2; ++c) {
            double v = at(H2 + r, H2 + c);
            if (GUARD) v = (r < nbr && c < nr) ? v : 0.0;
            bl[i][c] = v;
        }
    }
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const double g = rf.g[k];
        double uf[H2];
        team_gather<H, T>(rf.u[k], uf, tbuf, s);
        if (!first) {
            // left block: X += g u (u^T X)
#pragma unroll
            for (int c = 0; c < H; ++c) {
                double p = 0.0;
#pragma unroll
                for (int i = 0; i < RL; ++i) p += rf.u[k][i] * lf[i][c];
                const double f = g * group_sum<T>(p);
#pragma unroll
                for (int i = 0; i < RL; ++i) lf[i][c] += f * rf.u[k][i];
            }
        }
        // below block rows: X_B += g (X_B u) u^T
#pragma unroll
        for (int i = 0; i < RL; ++i) {
            double p = 0.0;
#pragma unroll
            for (int c = k; c < H2; ++c) p += bl[i][c] * uf[c];
            const double f = g * p;
#pragma unroll
            for (int c = k; c < H2; ++c) bl[i][c] += f * uf[c];
        }
        // diagonal block: p = g D u, w = p + (g/2)(u^T p) u, D += u w^T + w u^T
        double pl[RL];
        double upp = 0.0;
#pragma unroll
        for (int i = 0; i < RL; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int c = k; c < H2; ++c) acc += d[i][c] * uf[c];
            pl[i] = g * acc;
            upp += rf.u[k][i] * pl[i];
        }
        const double kk = 0.5 * g * group_sum<T>(upp);
        double wl[RL];
#pragma unroll
        for (int i = 0; i < RL; ++i) wl[i] = pl[i] + kk * rf.u[k][i];
        double wf[H2];
        team_gather<H, T>(wl, wf, tbuf + H2, s);
#pragma unroll
        for (int i = 0; i < RL; ++i)
#pragma unroll
            for (int c = 0; c < H2; ++c) d[i][c] += rf.u[k][i] * wf[c] + wl[i] * uf[c];
    }
    // write back the left block (j > 1), the lower part of the diagonal block
    // and the below block (the next chase's copy in registers supersedes it;
    // the last chase's is final)
#pragma unroll
    for (int i = 0; i < RL; ++i) {
        const int r = s + T * i;
        if (!GUARD || r < nr) {
            if (!first) {
#pragma unroll
                for (int c = 0; c < H; ++c) at(r, H + c) = lf[i][c];
            }
#pragma unroll
            for (int c = 0; c < H2; ++c)
                if (c <= r) col[H2 + c][r - c] = d[i][c];
        }
#pragma unroll
        for (int c = 0; c < H2; ++c)
            if (!GUARD || (r < nbr && c < nr)) at(H2 + r, H2 + c) = bl[i][c];
#pragma unroll
        for (int c = 0; c < H2; ++c) cy.b[i][c] = bl[i][c];
    }
}
