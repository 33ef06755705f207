// gfx950 kernels of libamfrw: payoff initialisation, the explicit operator of Sketch 1 fused with
// the AMFR-W stage combinations, the directional tridiagonal solves of Lemma lema:ls, tensor-product
// interpolation and the FP64 combination of component-grid values.
//
// Layout: every grid vector stores the inner nodes of all units back to back (unit offsets aligned
// to 64 elements); inside a unit axis 0 is fastest and M_i = 2^lv_i, so index decoding is shifts and
// masks.  Solution vectors hold W = Y - g, which vanishes on every lower (Dirichlet) face, so the
// time loop never evaluates the payoff: F(Y) = F0(W) + F(g) with F0 the zero-face operator and F(g)
// computed once per solve.
#include "amfrw_internal.h"

namespace amf {

// ------------------------------------------------------------------------------------------------
// Payoff g(T, F_1..F_{d-1}) in FP64 (Section 2): caplet tau_1 (F_1 - K)^+ or the swaption formula.
__device__ __forceinline__ double payoff_at(const ProbDev& P, int nr, const double* x)
{
    if (P.payoff == 0) {
        double v = P.tau[0] * (x[0] - P.K);
        return v > 0.0 ? v : 0.0;
    }
    double sum = 0.0, prod = 1.0;
    for (int i = 0; i < nr; ++i) {
        prod *= 1.0 + P.tau[i] * x[i];
        sum += P.tau[i] * (x[i] - P.K) / prod;
    }
    return sum > 0.0 ? sum : 0.0;
}

// Blocks are dealt round-robin to the XCDs; remap so that each XCD works on one contiguous eighth
// of the block range, keeping stencil halos (the neighbouring planes in the outer axes, read by the
// adjacent blocks) in that XCD's L2.  Schedule value 1 remaps the operator kernels only, 2 every
// streaming kernel (line blocks of uneven cost can then leave XCDs unevenly loaded).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb, int on)
{
    if (!on) return b;
    const int64_t x = b % NXCD, i = b / NXCD, q = nb / NXCD, r = nb % NXCD;
    return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ int find_unit(const UnitDev* units, int u, int64_t g)
{
    while (g >= units[u + 1].off) ++u;
    return u;
}

// ------------------------------------------------------------------------------------------------
// Per-node kernels: payoff g at every inner node, W = 0, and Y = W + g for read-back.
template <typename T, int D, int MODE>   // MODE 0: Y = g;  1: Y = 0;  2: Y = W + g
__global__ __launch_bounds__(NODE_BLOCK) void k_node(DevPlan P, const T* Win, T* Y)
{
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x, P.xcd == 2);
    const int64_t g = lb * NODE_BLOCK + threadIdx.x;
    if (g >= P.total) return;
    const int u = find_unit(P.units, P.blk_unit[lb], g);
    const UnitDev U = P.units[u];
    const int64_t loc = g - U.off;
    if (loc >= ((int64_t)1 << U.lsum)) {   // alignment padding
        Y[g] = T(0);
        return;
    }
    if constexpr (MODE == 1) {
        Y[g] = T(0);
    } else {
        const ProbDev& PR = P.probs[U.prob];
        double x[MAXD];
        int sh = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int M = 1 << U.lv[i];
            const int j = (int)((loc >> sh) & (M - 1)) + 1;
            x[i] = (double)j * (PR.xmax[i] / (double)M);
            sh += U.lv[i];
        }
        const double gv = payoff_at(PR, D - 1, x);
        if constexpr (MODE == 0) Y[g] = (T)gv;
        else Y[g] = (T)((double)Win[g] + gv);
    }
}

// ------------------------------------------------------------------------------------------------
// Sketch 1 at one inner node, fused with the stage combination selected by OP.
//
//   F(Y)_J = V^2 [ sum_i tdiff_i Delta2_i + sum_{i<k} C_ik tmix_i tmix_k X_ik
//                  + sum_{i=2..N-1} tmix_i (sum_{j=2..i} rho_ij tphi_j) D1_i ]
//
// with the raw differences Delta2 = Y+ - 2Y + Y-, X_ik = Y++ + Y-- - Y+- - Y-+, D1 = Y+ - Y-, the
// 1-D factors tdiff_i = alpha_i^2 F_i^(2 beta) / (2 h_i^2), tmix_i = alpha_i F_i^beta / (2 h_i),
// tphi_j = alpha_j Phi_beta(F_j, tau_j) of (coef_diff), (coef_mix), (coef_adv), tdiff_V =
// sigma^2 / (2 h_V^2), tmix_V = 1 / (2 h_V), C_ik = rho_ik (rates) or sigma phi_i (k = V).  At
// j_i = M_i the Neumann ghost Y_{J+E_i} = Y_{J-E_i} applies and the mixed and first differences are 0.
template <typename T, int D, int OP>
__global__ __launch_bounds__(NODE_BLOCK) void k_stencil(DevPlan P, StencilArgs A)
{
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x, P.xcd != 0);
    const int64_t g = lb * NODE_BLOCK + threadIdx.x;
    if (g >= P.total) return;
    const int u = find_unit(P.units, P.blk_unit[lb], g);
    const UnitDev U = P.units[u];
    const int64_t loc = g - U.off;
    if (loc >= ((int64_t)1 << U.lsum)) return;   // alignment padding
    const ProbDev& PR = P.probs[U.prob];
    const T* tab = (const T*)P.tab;
    const T* cst = tab + PR.cst;

    int j[D], M[D];
    int64_t E[D];
    {
        int sh = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            M[i] = 1 << U.lv[i];
            E[i] = (int64_t)1 << sh;
            j[i] = (int)((loc >> sh) & (M[i] - 1)) + 1;
            sh += U.lv[i];
        }
    }
    const T* X0 = (const T*)A.X0;
    const T* X1 = (const T*)A.X1;
    const T av = (T)A.a;
    auto X = [&](int64_t idx) -> T {
        if constexpr (OP == OP_STAGE2) return X0[idx] + av * X1[idx];
        else return X0[idx];
    };
    // value at j + si e_i + sk e_k when that node lies on a lower face
    auto face = [&](int i, int si, int k, int sk) -> T {
        if constexpr (OP != OP_F_PAYOFF) {
            return T(0);
        } else {
            double x[MAXD];
#pragma unroll
            for (int r = 0; r < D - 1; ++r) {
                const int jr = j[r] + (r == i ? si : 0) + (r == k ? sk : 0);
                x[r] = (double)jr * (PR.xmax[r] / (double)M[r]);
            }
            return (T)payoff_at(PR, D - 1, x);
        }
    };
    auto nb2 = [&](int i, int si, int k, int sk) -> T {
        if ((si < 0 && j[i] == 1) || (sk < 0 && j[k] == 1)) return face(i, si, k, sk);
        return X(g + si * E[i] + sk * E[k]);
    };

    const T c0 = X(g);
    T xm[D], xp[D], tmix[D], tphi[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        xm[i] = (j[i] == 1) ? face(i, -1, -1, 0) : X(g - E[i]);
        xp[i] = (j[i] == M[i]) ? xm[i] : X(g + E[i]);
    }
    const T* tV = tab + U.tab[D - 1];
    const int MV = M[D - 1];
    const T vsq = tV[j[D - 1] - 1];
    T acc = tV[MV] * (xp[D - 1] - T(2) * c0 + xm[D - 1]);
    tmix[D - 1] = tV[MV + 1];
    tphi[D - 1] = T(0);
#pragma unroll
    for (int i = 0; i < D - 1; ++i) {
        const T* ti = tab + U.tab[i];
        tmix[i] = ti[M[i] + j[i] - 1];
        tphi[i] = ti[2 * M[i] + j[i] - 1];
        acc += ti[j[i] - 1] * (xp[i] - T(2) * c0 + xm[i]);
    }
#pragma unroll
    for (int i = 0; i < D - 1; ++i) {
#pragma unroll
        for (int k = i + 1; k < D; ++k) {
            if (j[i] != M[i] && j[k] != M[k]) {
                const T xx = nb2(i, 1, k, 1) + nb2(i, -1, k, -1) - nb2(i, 1, k, -1) - nb2(i, -1, k, 1);
                const T cik = (k < D - 1) ? cst[CST_RHO + i * MAXD + k] : cst[CST_SPHI + i];
                acc += cik * tmix[i] * tmix[k] * xx;
            }
        }
    }
#pragma unroll
    for (int i = 1; i < D - 1; ++i) {
        if (j[i] != M[i]) {
            T s = T(0);
#pragma unroll
            for (int jj = 1; jj <= i; ++jj) s += cst[CST_RHO + i * MAXD + jj] * tphi[jj];
            acc += tmix[i] * s * (xp[i] - xm[i]);
        }
    }
    // nodes on a Dirichlet rate face (eq bound1_0) are boundary data: their row of F is null
    bool on_face = false;
#pragma unroll
    for (int i = 0; i < D - 1; ++i) on_face |= dir_face(PR.dirichlet, j[i], M[i]);
    const T F = on_face ? T(0) : vsq * acc;
    const T sc = A.scale_sel < 0 ? (T)A.scale : cst[A.scale_sel];
    T* W = (T*)A.W;
    const T* cG = (const T*)A.cG;
    if constexpr (OP == OP_F_PAYOFF || OP == OP_F_ZERO) {
        W[g] = sc * F;
    } else if constexpr (OP == OP_STAGE1) {
        W[g] = sc * (F + cG[g]);
    } else if constexpr (OP == OP_STAGE2) {
        const T* X2 = A.X2 ? (const T*)A.X2 : X1;
        W[g] = sc * (F + cG[g]) + (T)A.q * X2[g];
    } else {
        W[g] = T(2) * W[g] - X0[g] + sc * F;
    }
}

// ------------------------------------------------------------------------------------------------
// The same operator for the time loop (zero lower faces: W, K1 and the increments all vanish
// there), register-blocked: each thread evaluates R consecutive nodes of one axis-0 line, loading
// every neighbour row as an R-vector (plus the two axis-0 end values where a mixed (0,k) difference
// needs them) and sharing index decoding and the axis-1..d coefficient factors across the R nodes.
template <typename T, int R>
struct RowV {
    T v[R + 2];   // v[0] = left neighbour, v[1..R] = nodes, v[R+1] = right neighbour
};

template <typename T, int R>
__device__ __forceinline__ void load_vec(const T* p, T* dst)
{
    typedef T vt __attribute__((ext_vector_type(R)));
    const vt x = *(const vt*)p;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[r] = x[r];
}


template <typename T, int R>
__device__ __forceinline__ void store_vec(T* p, const T* v)
{
    typedef T vt __attribute__((ext_vector_type(R)));
    vt x;
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = v[r];
    *(vt*)p = x;
}

// Carry entering each segment of a line whose segments sit on consecutive threads of the block
// (segment `pos` of `nseg`, counted along the scan direction: forward = increasing rows, reversed =
// decreasing rows): inclusive scan of the affine maps c -> b + a c, one doubling round per
// __syncthreads_or, which also makes the round count block-uniform when the block holds lines of
// different lengths.  sh: 4*NODE_BLOCK entries of LDS (two ping-pong buffers of (a, b)).
template <typename T>
__device__ __forceinline__ T adjacent_carry(T a, T b, int pos, int nseg, bool rev, T* sh)
{
    const int tid = threadIdx.x;
    const int dir = rev ? 1 : -1;          // where the earlier segments of the scan sit
    T* buf = sh;
    buf[tid] = a;
    buf[NODE_BLOCK + tid] = b;
    int off = 1;
    while (__syncthreads_or(off < nseg)) {
        if (off < nseg && pos >= off) {
            const int at = tid + dir * off;
            const T pa = buf[at], pb = buf[NODE_BLOCK + at];
            b = b + a * pb;
            a = a * pa;
        }
        buf = (buf == sh) ? sh + 2 * NODE_BLOCK : sh;
        buf[tid] = a;
        buf[NODE_BLOCK + tid] = b;
        off <<= 1;
    }
    const T cin = pos > 0 ? buf[NODE_BLOCK + tid + dir] : T(0);
    __syncthreads();
    return cin;
}

// The same carry when every line's segments lie inside one wave (nseg <= 64; lines start at lane
// multiples of nseg): a doubling scan over lane shuffles, as many rounds as the wave's longest line
// needs, no LDS and no barrier.
template <typename T>
__device__ __forceinline__ T wave_carry(T a, T b, int pos, int nseg, bool rev)
{
    for (int off = 1; __any(off < nseg); off <<= 1) {
        const T pa = rev ? __shfl_down(a, off) : __shfl_up(a, off);
        const T pb = rev ? __shfl_down(b, off) : __shfl_up(b, off);
        if (off < nseg && pos >= off) {
            b = b + a * pb;
            a = a * pa;
        }
    }
    const T prev = rev ? __shfl_down(b, 1) : __shfl_up(b, 1);
    return pos > 0 ? prev : T(0);
}

// Axis-0 solve (I - nu dt A_1) x = v of the R rows r0..r0+R-1 this thread holds (segment s of the
// line's nseg = M0/R segments, consecutive threads), with the tabulated factors f = (inv, a inv,
// c') of the line: both Thomas recurrences from zero carries, carries scanned across the line's
// threads (in-wave shuffles unless a line of the block spans several waves), rows corrected.
// Every thread of the block must call it.
template <typename T, int R>
__device__ __forceinline__ void axis0_segment_solve(T* v, const T* f, int M0, int s, int nseg, bool live, T* sh)
{
    const bool wide = __syncthreads_or(nseg > 64);
    const int r0 = s * R;
    T y = T(0), mu = T(1);
    if (live) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T ai = f[M0 + r0 + k];
            y = v[k] * f[r0 + k] - ai * y;
            mu = -ai * mu;
            v[k] = y;
        }
    }
    const T yin = wide ? adjacent_carry<T>(mu, y, s, nseg, false, sh) : wave_carry<T>(mu, y, s, nseg, false);
    T x = T(0), nu = T(1);
    if (live) {
        T m = T(1);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            m = -f[M0 + r0 + k] * m;
            v[k] = v[k] + m * yin;
        }
#pragma unroll
        for (int k = R - 1; k >= 0; --k) {
            const T cp = f[2 * M0 + r0 + k];
            x = v[k] - cp * x;
            nu = -cp * nu;
            v[k] = x;
        }
    }
    const T xin = wide ? adjacent_carry<T>(nu, x, nseg - 1 - s, nseg, true, sh)
                       : wave_carry<T>(nu, x, nseg - 1 - s, nseg, true);
    if (live) {
        T n = T(1);
#pragma unroll
        for (int k = R - 1; k >= 0; --k) {
            n = -f[2 * M0 + r0 + k] * n;
            v[k] = v[k] + n * xin;
        }
    }
}

// Time-loop operator over R consecutive axis-0 nodes per thread.  FUSE: the block also solves the
// axis-0 systems of the first AMF factor on the values it produced (its lines lie whole inside the
// block: unit offsets are multiples of min(M0, 1024) and NODE_BLOCK*R >= M0) and writes them to
// A.S; the stage operators still write K^(0) to A.W (the refinement reads it), the refinement
// writes only the solved values.
template <typename T, int D, int OP, int R, bool FUSE>
__global__ __launch_bounds__(NODE_BLOCK) void k_stencil_vec(DevPlan P, StencilArgs A, int list)
{
    static_assert(OP == OP_STAGE1 || OP == OP_STAGE2 || OP == OP_REFINE, "zero-face operators only");
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x, P.xcd != 0);
    // fused: dense blocks over the whole vector (one R for the plan); else the block list of one
    // axis-1 line class (each unit at R = min(stencil_nodes, M_1))
    int64_t g, gend;
    int32_t u0;
    if constexpr (FUSE) {
        g = (lb * NODE_BLOCK + threadIdx.x) * R;
        gend = P.total;
        u0 = g < P.total ? P.blk_unit_r[r_index(R)][lb] : 0;
    } else {
        const VecBlk B = P.vblk[P.vblk_off[list] + lb];
        g = B.g0 + (int64_t)threadIdx.x * R;
        gend = B.gend;
        u0 = B.unit;
    }
    bool live = g < gend;
    if constexpr (!FUSE) {
        if (!live) return;
    }
    int u = 0;
    int64_t loc = 0;
    if (live) {
        u = find_unit(P.units, u0, g);
        loc = g - P.units[u].off;
        live = loc < ((int64_t)1 << P.units[u].lsum);     // else alignment padding
    }
    if constexpr (!FUSE) {
        if (!live) return;
    }
    T o[R];
#pragma unroll
    for (int r = 0; r < R; ++r) o[r] = T(0);
    // the operator itself is written out in the kernel body (an extracted device function costs
    // ~50 VGPRs here: its lambdas lose track of which values are wave-uniform)
    if (live) {
        const UnitDev U = P.units[u];
        const ProbDev& PR = P.probs[U.prob];
        const T* tab = (const T*)P.tab;
        const T* cst = tab + PR.cst;

        int j[D], M[D];
        int64_t E[D];
        {
            int sh = 0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                M[i] = 1 << U.lv[i];
                E[i] = (int64_t)1 << sh;
                j[i] = (int)((loc >> sh) & (M[i] - 1)) + 1;   // j[0] = first of the R nodes
                sh += U.lv[i];
            }
        }
        const T* X0 = (const T*)A.X0;
        const T* X1 = (const T*)A.X1;
        const T av = (T)A.a;
        const bool has_left = j[0] > 1, has_right = j[0] + R - 1 < M[0];
        const int lane = threadIdx.x & 63;
        auto X = [&](int64_t idx) -> T {
            if constexpr (OP == OP_STAGE2) return X0[idx] + av * X1[idx];
            else return X0[idx];
        };
        // v[1..R]: the row of R nodes at offset o (0 where !ok).  With `ends` (wave-uniform: every
        // active lane must reach the shuffles) also v[0], v[R+1]: the axis-0 neighbours, taken from
        // the adjacent lanes' rows (lanes hold consecutive R-node chunks), loaded only by the lanes
        // at the wave's edges, 0 on the lower face and beyond the line's end.
        auto load_row = [&](int64_t o, bool ends, bool ok, T* v) {
            if (ok) {
                load_vec<T, R>(X0 + g + o, v + 1);
                if constexpr (OP == OP_STAGE2) {
                    T w[R];
                    load_vec<T, R>(X1 + g + o, w);
#pragma unroll
                    for (int r = 0; r < R; ++r) v[1 + r] += av * w[r];
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[1 + r] = T(0);
            }
            v[0] = T(0);
            v[R + 1] = T(0);
            if (ends) {
                const T lv = __shfl_up(v[R], 1);
                const T rv = __shfl_down(v[1], 1);
                if (ok && has_left) v[0] = lane == 0 ? X(g + o - 1) : lv;
                if (ok && has_right) v[R + 1] = lane == 63 ? X(g + o + R) : rv;
            }
        };

        T c[R + 2];
        load_row(0, true, true, c);
        T acc[R];
        // axis 0: second differences with the Neumann ghost at j_0 = M_0; coefficients per node
        const T* t0 = tab + U.tab[0];
        T tmix0[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int jr = j[0] + r;
            const T xm = c[r];
            const T xp = (jr == M[0]) ? xm : c[r + 2];
            acc[r] = t0[jr - 1] * (xp - T(2) * c[r + 1] + xm);
            tmix0[r] = t0[M[0] + jr - 1];
        }
        // axes 1..D-1: rows at -E_k and +E_k (reflected at j_k = M_k), shared coefficients
        T tmix[D], tphi[D];
        const T* tV = tab + U.tab[D - 1];
        const int MV = M[D - 1];
        const T vsq = tV[j[D - 1] - 1];
#pragma unroll
        for (int k = 1; k < D; ++k) {
            T rm[R + 2], rp[R + 2];
            const bool up_ok = j[k] != M[k];
            load_row(-E[k], true, j[k] > 1, rm);
            load_row(E[k], true, up_ok, rp);
            if (!up_ok) {
#pragma unroll
                for (int r = 0; r < R + 2; ++r) rp[r] = rm[r];
            }
            T td;
            if (k < D - 1) {
                const T* tk = tab + U.tab[k];
                td = tk[j[k] - 1];
                tmix[k] = tk[M[k] + j[k] - 1];
                tphi[k] = tk[2 * M[k] + j[k] - 1];
            } else {
                td = tV[MV];
                tmix[k] = tV[MV + 1];
                tphi[k] = T(0);
            }
            // advection on axes 1..D-2 (paper axes 2..N-1), zero on the upper face
            T adv = T(0);
            if (k < D - 1 && up_ok) {
#pragma unroll
                for (int jj = 1; jj <= k; ++jj) adv += cst[CST_RHO + k * MAXD + jj] * tphi[jj];
                adv *= tmix[k];
            }
            const T c0k = (k < D - 1) ? cst[CST_RHO + 0 * MAXD + k] : cst[CST_SPHI + 0];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                acc[r] += td * (rp[r + 1] - T(2) * c[r + 1] + rm[r + 1]);
                if (k < D - 1 && up_ok) acc[r] += adv * (rp[r + 1] - rm[r + 1]);
                // mixed (0, k): zero when either node index is on its upper face
                if (up_ok && (j[0] + r) != M[0]) {
                    const T xx = rp[r + 2] + rm[r] - rp[r] - rm[r + 2];
                    acc[r] += c0k * tmix0[r] * tmix[k] * xx;
                }
            }
        }
        // mixed (i, k), 1 <= i < k: four diagonal rows of R nodes
#pragma unroll
        for (int i = 1; i < D - 1; ++i) {
#pragma unroll
            for (int k = i + 1; k < D; ++k) {
                if (j[i] != M[i] && j[k] != M[k]) {
                    T pp[R + 2], mm[R + 2], pm[R + 2], mp[R + 2];
                    load_row(E[i] + E[k], false, true, pp);
                    load_row(-E[i] - E[k], false, j[i] > 1 && j[k] > 1, mm);
                    load_row(E[i] - E[k], false, j[k] > 1, pm);
                    load_row(-E[i] + E[k], false, j[i] > 1, mp);
                    const T cik = ((k < D - 1) ? cst[CST_RHO + i * MAXD + k] : cst[CST_SPHI + i]) * tmix[i] * tmix[k];
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r] += cik * (pp[r + 1] + mm[r + 1] - pm[r + 1] - mp[r + 1]);
                }
            }
        }
        const T sc = A.scale_sel < 0 ? (T)A.scale : cst[A.scale_sel];
        const T* W = (const T*)A.W;
        const T* cG = (const T*)A.cG;
        T e[R];
        if constexpr (OP == OP_STAGE1 || OP == OP_STAGE2) load_vec<T, R>(cG + g, e);
        if constexpr (OP == OP_REFINE) {
            load_vec<T, R>(W + g, e);     // K^(0)
        }
        T q1[R];
        if constexpr (OP == OP_STAGE2) load_vec<T, R>((A.X2 ? (const T*)A.X2 : X1) + g, q1);
        // Dirichlet rate faces (eq bound1_0): rows of boundary data, F = 0 there
        const bool dirp = PR.dirichlet != 0;
        bool rowface = false;
#pragma unroll
        for (int k = 1; k < D - 1; ++k) rowface |= dir_face(dirp, j[k], M[k]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const T F = (rowface || dir_face(dirp, j[0] + r, M[0])) ? T(0) : vsq * acc[r];
            if constexpr (OP == OP_STAGE1) o[r] = sc * (F + e[r]);
            else if constexpr (OP == OP_STAGE2) o[r] = sc * (F + e[r]) + (T)A.q * q1[r];
            else o[r] = T(2) * e[r] - c[r + 1] + sc * F;
        }
        if (!FUSE || OP != OP_REFINE) store_vec<T, R>((T*)A.W + g, o);
    }
    if constexpr (FUSE) {
        __shared__ T sh[4 * NODE_BLOCK];
        int s = 0, nseg = 1, M0 = R;
        const T* f = (const T*)P.fac;
        if (live) {
            const UnitDev& U = P.units[u];
            int SV = 0;
#pragma unroll
            for (int k = 0; k < D - 1; ++k) SV += U.lv[k];
            M0 = 1 << U.lv[0];
            s = (int)(loc & (M0 - 1)) / R;
            nseg = M0 / R;
            const int64_t jv = (loc >> SV) & ((1 << U.lv[D - 1]) - 1);
            f += (int64_t)U.fac[0] + (int64_t)A.run * P.fac_run_stride + jv * 3 * M0;
        }
        axis0_segment_solve<T, R>(o, f, M0, s, nseg, live, sh);
        if (live) store_vec<T, R>((T*)A.S + g, o);
    }
}

// ------------------------------------------------------------------------------------------------
// The time-loop operator in its plane-tiled form (amfrw_march.h): one block per (unit, tile of the
// plane axes, range of V planes); the neighbour values come from a ring of LDS plane slots.  Global
// traffic goes through buffer loads and stores on one V plane of the unit at a time: a fetch whose
// offset lies beyond the plane (the zero halo elements, every element of plane 0) returns 0.
template <typename T>
struct GpuMem {
    using bits = typename std::conditional<sizeof(T) == 8, unsigned int __attribute__((ext_vector_type(2))),
                                           unsigned int>::type;
    struct Plane {
        __amdgpu_buffer_rsrc_t r;
    };
    T* lds;
    __device__ __forceinline__ Plane plane(const T* p, int64_t base, int64_t n) const
    {
        return {__builtin_amdgcn_make_buffer_rsrc((void*)(p + base), (short)0, (int)(n * (int64_t)sizeof(T)),
                                                  0x00020000)};
    }
    __device__ __forceinline__ T pld(const Plane& h, uint32_t b) const
    {
        if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(h.r, b, 0, 0));
        else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(h.r, b, 0, 0));
    }
    __device__ __forceinline__ void pst(const Plane& h, uint32_t b, T v) const
    {
        if constexpr (sizeof(T) == 8) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bits, v), h.r, b, 0, 0);
        else __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(bits, v), h.r, b, 0, 0);
    }
    __device__ __forceinline__ T tab(const T* p, int i) const { return p[i]; }
    __device__ __forceinline__ T sr(int i) const { return lds[i]; }
    __device__ __forceinline__ void sw(int i, T v) const { lds[i] = v; }
};

// DPP row shifts inside rows of 16 lanes: row_shr:K gives lane i the value of lane i - K of its row,
// row_shl:K that of lane i + K (0 from outside the row).  Register moves only.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

constexpr int DPP_ROW_SHL = 0x100, DPP_ROW_SHR = 0x110;

// Solves a tridiagonal system of M <= 16 rows held one row per lane in M consecutive lanes (the
// group aligned inside a 16-lane row; r = the lane's row) with the tabulated Thomas factors of its
// row (Lemma lema:ls): forward d'_r = g_r inv_r - (a inv)_r d'_{r-1}, backward x_r = d'_r -
// c'_r x_{r+1}.  Each recurrence is affine, y_r = alpha_r + beta_r y_{r -/+ 1}, and is evaluated by
// a scan of log2(M) steps, composing the maps of lanes K apart.
template <int K, typename T>
__device__ __forceinline__ void scan_down(T& al, T& be, int r, int M)
{
    if (K < M) {
        const T pa = dpp_move<DPP_ROW_SHR + K>(al), pb = dpp_move<DPP_ROW_SHR + K>(be);
        if (r >= K) {
            al = al + be * pa;
            be = be * pb;
        }
    }
}

template <int K, typename T>
__device__ __forceinline__ void scan_up(T& al, T& be, int r, int M)
{
    if (K < M) {
        const T na = dpp_move<DPP_ROW_SHL + K>(al), nb = dpp_move<DPP_ROW_SHL + K>(be);
        if (r + K < M) {
            al = al + be * na;
            be = be * nb;
        }
    }
}

template <typename T>
__device__ __forceinline__ T row_solve(T g, T inv, T ainv, T cp, int r, int M)
{
    T al = g * inv, be = -ainv;
    scan_down<1>(al, be, r, M);
    scan_down<2>(al, be, r, M);
    scan_down<4>(al, be, r, M);
    scan_down<8>(al, be, r, M);
    T bl = al, bb = -cp;
    scan_up<1>(bl, bb, r, M);
    scan_up<2>(bl, bb, r, M);
    scan_up<4>(bl, bb, r, M);
    scan_up<8>(bl, bb, r, M);
    return bl;
}

// One block.  Per step: plane j_V + 2 (loaded MARCH_DEPTH steps before) into its slot, plane
// j_V + 2 + MARCH_DEPTH and the next node's stage values loaded, plane j_V computed and stored.  Loads
// are issued in the order they are waited for, so no wait covers a load issued later in the same
// step, and each plane's loads have MARCH_DEPTH steps to arrive.
template <typename T, int D, int OP, class Sh>
__device__ __forceinline__ void march_block(const DevPlan& P, const StencilArgs& A, const MarchBlk& B, T* smem)
{
    constexpr int NPF = Sh::NPF;
    constexpr int DP = MARCH_DEPTH;
    GpuMem<T> m{smem};
    const UnitDev& U = P.units[B.unit];
    MarchGeo<D> G;
    march_geo<D>(U.lv, U.off, B, G);
    const ProbDev& PR = P.probs[U.prob];
    const T* tab = (const T*)P.tab;
    const T* cst = tab + PR.cst;
    const int tid = threadIdx.x;
    MarchThr<T, D, NPF> t;
    march_thread<T, D, Sh>(G, tid, t);
    march_coefs<T, D>(G, U.tab, tab, cst, t, m);
    march_face<T, D>(PR.dirichlet, t);
    const T* X0 = (const T*)A.X0;
    const T* X1 = (const T*)A.X1;
    const T av = (T)A.a;
    const T* tV = tab + U.tab[D - 1];
    const T sc = A.scale_sel < 0 ? (T)A.scale : cst[A.scale_sel];
    const T qv = (T)A.q;
    const int MV = G.M[D - 1];
    const T tdV = tV[MV];
    const int last = min(MV, G.v0 + G.vn + 1);            // last plane the block reads
    const T* cE = OP == OP_REFINE ? (const T*)A.W : (const T*)A.cG;
    const T* X2 = A.X2 ? (const T*)A.X2 : X1;
    T* W = (T*)A.W;
    const bool act = t.active;
    // fused axis-1 solve (uniform over the block): the tile rows are whole axis-1 lines
    const bool fz = march_fused<D>(G, A.S != nullptr);
    T* Sv = (T*)A.S;
    const T* fa0 = (const T*)P.fac + (int64_t)A.run * P.fac_run_stride + U.fac[0];
    // the values the stage combination needs at this thread's node of plane jv
    auto centre = [&](int jv, T (&e)[2], bool live) {
        const int64_t b = march_plane_base<D>(G, jv), n = live ? march_plane_len<D>(G, jv) : 0;
        e[0] = m.pld(m.plane(cE, b, n), t.gob);               // K^(0) for the refinement
        e[1] = OP == OP_STAGE2 ? m.pld(m.plane(X2, b, n), t.gob) : T(0);
    };
    march_vsq<T, D, Sh>(G, tid, tV, m);
    // planes v0 .. v0 + 2 into their slots (plane 0 is the lower face: zeros), planes v0 + 3 ..
    // v0 + 2 + DP in flight: plane v0 + i goes to register set i mod DP, and the set is stashed
    // before it is loaded again
    MarchPf<T, OP, NPF> pf[DP];
#pragma unroll
    for (int i = 0; i < 3 + DP; ++i) {
        const int p = G.v0 + i;
        if (i >= DP && p - DP <= last) march_stash<T, D, Sh>(G, tid, p - DP, pf[(i - DP) % DP], av, m);
        march_fetch<T, D, OP>(G, p, X0, X1, t, pf[i % DP], m, p <= last);
    }
    T ce[2][2] = {};
    centre(G.v0 + 1, ce[0], true);
    __syncthreads();
    // crosses of the planes v0 and v0 + 1 (stashed above); each step reads that of plane jv + 1
    constexpr int NX = MarchX<D>::N;
    T xw[3][NX];
    if (act) {
        march_cross<T, D, Sh>(G, t, G.v0, xw[0], m);
        march_cross<T, D, Sh>(G, t, G.v0 + 1, xw[1], m);
    }
    // step s = position k in a period of 6 computes plane v0 + s from the crosses of planes jv - 1
    // and jv (register sets k and k + 1 mod 3) and jv + 1 (read into set k + 2 mod 3) and from the
    // stage values in set k mod 2, and loads those of the next plane into the other set.  The
    // register sets rotate, so no value is copied between steps (a copy of a loaded value would wait
    // for its load).  Every step issues the same global loads (empty ranges past the block's planes),
    // so each wait covers exactly the loads of the steps before.
    auto step = [&](auto K, int s) {
        constexpr int k = decltype(K)::value;
        const int jv = G.v0 + s;
        MarchPf<T, OP, NPF>& q = pf[(k + 1) % DP];          // holds plane jv + 2
        // plane jv + 2 goes into the slot of plane jv - 2, which no thread has read since the
        // barrier before the previous step
        if (jv + 2 <= last) march_stash<T, D, Sh>(G, tid, jv + 2, q, av, m);
        // factors of the fused solve: issued before the plane prefetch, so that waiting for them does
        // not wait for the prefetch
        T finv = T(0), fainv = T(0), fcp = T(0);
        if (fz && act) {
            const T* f = fa0 + march_fac_at<T, D>(G, jv, t);
            finv = f[0];
            fainv = f[G.M[0]];
            fcp = f[2 * G.M[0]];
        }
        march_fetch<T, D, OP>(G, jv + 2 + DP, X0, X1, t, q, m, jv + 2 + DP <= last);
        centre(jv + 1, ce[(k + 1) % 2], s < G.vn);
        const T vsq = march_vsq_of<T, D, Sh>(G, s, m);
        T o = T(0);
        if (act) {
            if (jv < MV) march_cross<T, D, Sh>(G, t, jv + 1, xw[(k + 2) % 3], m);   // uniform over the block
            const T F = march_F<T, D, Sh>(G, t, jv, vsq, tdV, xw[k % 3], xw[(k + 1) % 3], xw[(k + 2) % 3], m);
            const T c0_ = ce[k % 2][0], c1_ = ce[k % 2][1];
            if constexpr (OP == OP_STAGE1) o = sc * (F + c0_);
            else if constexpr (OP == OP_STAGE2) o = sc * (F + c0_) + qv * c1_;
            else o = T(2) * c0_ - xw[(k + 1) % 3][0] + sc * F;
            // the refinement's unsolved value is not read again when its line is solved here
            if (!(fz && OP == OP_REFINE)) m.pst(m.plane(W, march_plane_base<D>(G, jv), march_plane_len<D>(G, jv)), t.gob, o);
        }
        if (fz) {                                   // every lane takes part in the row scans
            const T x = row_solve<T>(o, finv, fainv, fcp, t.j[0] - 1, G.M[0]);
            if (act) m.pst(m.plane(Sv, march_plane_base<D>(G, jv), march_plane_len<D>(G, jv)), t.gob, x);
        }
        __syncthreads();
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;
    for (int s = 1; s <= G.vn; s += 6) {
        step(I0{}, s);
        if (s + 1 <= G.vn) step(I1{}, s + 1);
        if (s + 2 <= G.vn) step(I2{}, s + 2);
        if (s + 3 <= G.vn) step(I3{}, s + 3);
        if (s + 4 <= G.vn) step(I4{}, s + 4);
        if (s + 5 <= G.vn) step(I5{}, s + 5);
    }
}

template <typename T, int D, int OP>
__global__ __launch_bounds__(MARCH_THREADS) void k_march(DevPlan P, StencilArgs A)
{
    static_assert(MARCH_FUSE_LM == SHORT_LM, "the fused units are those of the short axis-1 sweep");
    static_assert(OP == OP_STAGE1 || OP == OP_STAGE2 || OP == OP_REFINE, "zero-face operators only");
    extern __shared__ __align__(16) unsigned char march_smem[];
    const MarchBlk B = (P.xcd ? P.march_blk_x : P.march_blk)[blockIdx.x];
    if (B.vn == 0) return;                                  // padding of the XCD-ordered table
    march_dispatch<D>(B.shape, [&](auto sh) { march_block<T, D, OP, decltype(sh)>(P, A, B, (T*)march_smem); });
}

// ------------------------------------------------------------------------------------------------
// Directional solves (I - nu dt A_i) x = G (Lemma lema:ls): rows r = 0..M-1 with delta_r =
// d_i / h_i^2, diagonal 1 + 2 nu dt delta_r, super-diagonal -nu dt delta_r (none in the last row),
// sub-diagonal -nu dt delta_r (none in the first row, doubled in the last row: Neumann ghost).
// The matrix of a line depends only on (problem, axis, M_axis, j_V) and dt, so strided axes use
// Thomas factors (inv_r = 1/pivot_r, a_r inv_r, c'_r) tabulated once per plan in FP64.

// Grid vectors are streamed once per sweep: in FP64 loads and stores carry the non-temporal hint
// (measured faster there, slower in FP32).
template <typename T>
struct elem_of { using type = T; };
template <typename T, int N>
struct elem_of<T __attribute__((ext_vector_type(N)))> { using type = T; };

template <typename T>
__device__ __forceinline__ T ld_stream(const T* p)
{
    if constexpr (sizeof(typename elem_of<T>::type) == 8) return __builtin_nontemporal_load(p);
    else return *p;
}

template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v)
{
    if constexpr (sizeof(typename elem_of<T>::type) == 8) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <typename T, int EPI>
__device__ __forceinline__ void sweep_store(const SweepArgs& A, int64_t idx, T x)
{
    if constexpr (EPI == EPI_STORE) {
        st_stream((T*)A.out + idx, x);
    } else {
        T* W = (T*)A.out;
        st_stream(W + idx, ld_stream(W + idx) + (T)A.b1 * ld_stream((const T*)A.K1 + idx) + (T)A.b2 * x);
    }
}

struct Strided {
    int64_t base;     // element index of row 0
    int64_t stride;   // E_axis
    int64_t fac;      // factor block of this line: inv[M], ainv[M], cp[M]
};

__device__ __forceinline__ Strided strided_geom(const DevPlan& P, const UnitDev& U, int axis,
                                                int64_t line, int lm, int run)
{
    const int D = P.d;
    int S = 0, SV = 0;
    for (int k = 0; k < axis; ++k) S += U.lv[k];
    for (int k = 0; k < D - 1; ++k) SV += U.lv[k];
    const int64_t E = (int64_t)1 << S;
    const int64_t lo = line & (E - 1), hi = line >> S;
    const int64_t loc0 = lo + (hi << (S + lm));
    Strided L;
    L.base = U.off + loc0;
    L.stride = E;
    L.fac = (int64_t)U.fac[axis] + (int64_t)run * P.fac_run_stride;
    if (axis < D - 1) {
        const int MV = 1 << U.lv[D - 1];
        const int64_t jv = (loc0 >> SV) & (MV - 1);
        L.fac += jv * 3 * ((int64_t)1 << lm);
    }
    return L;
}

// Strided axis, line kept in VGPRs: one thread per line, lanes on consecutive lines (coalesced).
template <typename T, int LM, int EPI>
__device__ __forceinline__ void sweep_strided_reg(const DevPlan& P, const SweepArgs& A, const Strided& L)
{
    constexpr int M = 1 << LM;
    const T* in = (const T*)A.in;
    const T* f = (const T*)P.fac + L.fac;
    T dp[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const T G = ld_stream(in + L.base + r * L.stride);
        dp[r] = (r == 0) ? G * f[0] : G * f[r] - f[M + r] * dp[r - 1];
    }
    T x = dp[M - 1];
    sweep_store<T, EPI>(A, L.base + (int64_t)(M - 1) * L.stride, x);
#pragma unroll
    for (int r = M - 2; r >= 0; --r) {
        x = dp[r] - f[2 * M + r] * x;
        sweep_store<T, EPI>(A, L.base + r * L.stride, x);
    }
}

// The same for V adjacent lines per thread (V * sizeof(T) = 16 B): one vector load and store per
// row for all V lines, which share the factor table (same j_V).  base and stride are multiples of V.
template <typename T, int LM, int EPI, int V>
__device__ __forceinline__ void sweep_strided_regv(const DevPlan& P, const SweepArgs& A, const Strided& L)
{
    typedef T vt __attribute__((ext_vector_type(V)));
    constexpr int M = 1 << LM;
    const T* in = (const T*)A.in;
    const T* f = (const T*)P.fac + L.fac;
    vt dp[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const vt G = *(const vt*)(in + L.base + r * L.stride);
        if (r == 0) dp[r] = G * f[0];
        else dp[r] = G * f[r] - f[M + r] * dp[r - 1];
    }
    vt x = dp[M - 1];
    auto put = [&](int64_t idx, vt v) {
        if constexpr (EPI == EPI_STORE) {
            *(vt*)((T*)A.out + idx) = v;         // (measured: plain faster than non-temporal here)
        } else {
            vt* W = (vt*)((T*)A.out + idx);
            st_stream(W, ld_stream(W) + (T)A.b1 * ld_stream((const vt*)((const T*)A.K1 + idx)) + (T)A.b2 * v);
        }
    };
    put(L.base + (int64_t)(M - 1) * L.stride, x);
#pragma unroll
    for (int r = M - 2; r >= 0; --r) {
        x = dp[r] - f[2 * M + r] * x;
        put(L.base + r * L.stride, x);
    }
}

template <typename T, int V>
struct lane_vec {
    typedef T __attribute__((ext_vector_type(V))) type;
};
template <typename T>
struct lane_vec<T, 1> {
    typedef T type;
};

// Two line slots per thread (lines of at most 2^PAIR_LM points, where one slot leaves too few loads
// in flight): the rows of both slots are loaded before either is solved and stored.  `two` is
// false when the block has no second slot for this thread; the second slot then repeats the first
// and is not stored.  The slots never overlap, so the in-place sweep stays exact.
template <typename T, int LM, int EPI, int V>
__device__ __forceinline__ void sweep_strided_pair(const DevPlan& P, const SweepArgs& A, const Strided& L1,
                                                   const Strided& L2, bool two)
{
    typedef typename lane_vec<T, V>::type vt;
    constexpr int M = 1 << LM;
    const T* in = (const T*)A.in;
    const T* f1 = (const T*)P.fac + L1.fac;
    const T* f2 = (const T*)P.fac + L2.fac;
    auto get = [&](int64_t idx) -> vt {
        if constexpr (V == 1) return ld_stream(in + idx);
        else return *(const vt*)(in + idx);
    };
    auto put = [&](int64_t idx, vt v) {
        if constexpr (V == 1) {
            sweep_store<T, EPI>(A, idx, v);
        } else if constexpr (EPI == EPI_STORE) {
            *(vt*)((T*)A.out + idx) = v;
        } else {
            vt* W = (vt*)((T*)A.out + idx);
            st_stream(W, ld_stream(W) + (T)A.b1 * ld_stream((const vt*)((const T*)A.K1 + idx)) + (T)A.b2 * v);
        }
    };
    vt d1[M], d2[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        d1[r] = get(L1.base + r * L1.stride);
        d2[r] = get(L2.base + r * L2.stride);
    }
#pragma unroll
    for (int r = 0; r < M; ++r) {
        if (r == 0) {
            d1[0] = d1[0] * f1[0];
            d2[0] = d2[0] * f2[0];
        } else {
            d1[r] = d1[r] * f1[r] - f1[M + r] * d1[r - 1];
            d2[r] = d2[r] * f2[r] - f2[M + r] * d2[r - 1];
        }
    }
#pragma unroll
    for (int r = M - 2; r >= 0; --r) {
        d1[r] = d1[r] - f1[2 * M + r] * d1[r + 1];
        d2[r] = d2[r] - f2[2 * M + r] * d2[r + 1];
    }
#pragma unroll
    for (int r = M - 1; r >= 0; --r) {
        put(L1.base + r * L1.stride, d1[r]);
        if (two) put(L2.base + r * L2.stride, d2[r]);
    }
}

// Short strided lines (up to 2^SHORT_LM rows): one thread per B.vec adjacent lines (1, or
// VW = 16 B / sizeof(T) when all the block's units allow it: one vector load and store per row),
// and per B.slots such slots (two for lines of at most 2^PAIR_LM points).
template <typename T, int EPI>
__global__ __launch_bounds__(LINE_BLOCK) void k_sweep_strided(DevPlan P, SweepArgs A, int axis, int64_t blk0)
{
    constexpr int VW = 16 / (int)sizeof(T);
    const SweepBlk B = P.ax_blk[axis][blk0 + xcd_block(blockIdx.x, gridDim.x, P.xcd == 2)];
    const int64_t gl = B.line_start + (int64_t)threadIdx.x * B.vec;
    if (gl >= B.line_end) return;
    const int64_t* lo = P.ax_line_off[axis];
    int k = B.k_start;
    if constexpr (EPI == EPI_STORE) {
        if (B.slots == 2) {                     // block-uniform; lines of at most 2^PAIR_LM points, axes 2..N-1
            while (gl >= lo[k + 1]) ++k;
            const Strided L = strided_geom(P, P.units[P.ax_units[axis][k]], axis, gl - lo[k], B.lm, A.run);
            const int64_t gl2 = gl + (int64_t)LINE_BLOCK * B.vec;
            const bool two = gl2 < B.line_end;
            Strided L2 = L;
            if (two) {
                while (gl2 >= lo[k + 1]) ++k;
                L2 = strided_geom(P, P.units[P.ax_units[axis][k]], axis, gl2 - lo[k], B.lm, A.run);
            }
            static_assert(PAIR_LM <= 2, "pair cases below");
            if (B.vec == 1) {
                switch (B.lm) {
                case 0: sweep_strided_pair<T, 0, EPI, 1>(P, A, L, L2, two); break;
                case 1: sweep_strided_pair<T, 1, EPI, 1>(P, A, L, L2, two); break;
                case 2: sweep_strided_pair<T, 2, EPI, 1>(P, A, L, L2, two); break;
                default: break;
                }
            } else {
                switch (B.lm) {
                case 0: sweep_strided_pair<T, 0, EPI, VW>(P, A, L, L2, two); break;
                case 1: sweep_strided_pair<T, 1, EPI, VW>(P, A, L, L2, two); break;
                case 2: sweep_strided_pair<T, 2, EPI, VW>(P, A, L, L2, two); break;
                default: break;
                }
            }
            return;
        }
    }
    // one slot (the update form runs on the last axis only, whose blocks are never paired)
    while (gl >= lo[k + 1]) ++k;
    const UnitDev U = P.units[P.ax_units[axis][k]];
    const Strided L = strided_geom(P, U, axis, gl - lo[k], B.lm, A.run);
    if (B.vec == 1) {                       // block-uniform
        switch (B.lm) {
        case 0: sweep_strided_reg<T, 0, EPI>(P, A, L); break;
        case 1: sweep_strided_reg<T, 1, EPI>(P, A, L); break;
        case 2: sweep_strided_reg<T, 2, EPI>(P, A, L); break;
        case 3: sweep_strided_reg<T, 3, EPI>(P, A, L); break;
        case 4: sweep_strided_reg<T, 4, EPI>(P, A, L); break;
        default: break;   // longer classes go to k_sweep_strided_long
        }
    } else {
        switch (B.lm) {
        case 0: sweep_strided_regv<T, 0, EPI, VW>(P, A, L); break;
        case 1: sweep_strided_regv<T, 1, EPI, VW>(P, A, L); break;
        case 2: sweep_strided_regv<T, 2, EPI, VW>(P, A, L); break;
        case 3: sweep_strided_regv<T, 3, EPI, VW>(P, A, L); break;
        case 4: sweep_strided_regv<T, 4, EPI, VW>(P, A, L); break;
        default: break;
        }
    }
}

// Inclusive scan, in segment order (reversed when `rev`), of the affine maps c -> b + a c of the
// segments of each line slot (a slot is one line, or V adjacent lines as one vector T); returns the
// map of all segments before this one applied to 0, i.e. the carry entering this segment.
// sh: 4*SEG_BLOCK entries of LDS (two ping-pong buffers of (a, b), segment-major), so each
// doubling round needs one barrier.
template <typename T>
__device__ __forceinline__ T segment_carry(T a, T b, int seg, int nseg, int line, int lines, bool rev, T* sh)
{
    const int s = rev ? nseg - 1 - seg : seg;
    const int at = s * lines + line;
    T* buf = sh;
    buf[at] = a;
    buf[SEG_BLOCK + at] = b;
    __syncthreads();
    for (int off = 1; off < nseg; off <<= 1) {
        if (s >= off) {
            const T pa = buf[at - off * lines], pb = buf[SEG_BLOCK + at - off * lines];
            b = b + a * pb;        // earlier segments first: b + a (pb + pa c)
            a = a * pa;
        }
        buf = (buf == sh) ? sh + 2 * SEG_BLOCK : sh;
        buf[at] = a;
        buf[SEG_BLOCK + at] = b;
        __syncthreads();
    }
    const T cin = s > 0 ? buf[SEG_BLOCK + at - lines] : T{};
    __syncthreads();           // the buffers are reused by the next scan
    return cin;
}

// Scalar or V-wide (ext_vector) element of the long-line solver.
// Long strided line split into nseg = M/S segments of S = seg_rows consecutive rows, one per thread,
// kept in VGPRs; with V > 1 the thread carries V adjacent lines (same factors) as one vector per
// row.  Both Thomas recurrences are first order and linear, y_r = g_r inv_r - ainv_r y_{r-1} and
// x_r = y_r - cp_r x_{r+1}: each thread runs them over its rows from a zero carry, the segments'
// affine end maps are scanned in LDS to give every segment its true carry, and the rows are
// corrected by the carry times the running product of the multipliers.  Every element is read and
// written once, by the same thread (in-place safe).  All threads of the block must call it
// (barriers); `live` is false for threads without a line.
template <typename T, int EPI, int V>
__device__ __forceinline__ void sweep_strided_seg(const DevPlan& P, const SweepArgs& A, const Strided& L, int lm,
                                                  bool live, int seg, int nseg, int line, int lines,
                                                  typename lane_vec<T, V>::type* sh)
{
    typedef typename lane_vec<T, V>::type vt;
    const int M = 1 << lm;
    constexpr int SSEG = seg_rows((int)sizeof(T), V);
    const int r0 = seg * SSEG;
    const T* f = (const T*)P.fac + (live ? L.fac : 0);
    const vt one = vt{} + T(1);
    vt v[SSEG];
    vt y{}, mu = one;
    if (live) {
        const T* in = (const T*)A.in;
#pragma unroll
        for (int k = 0; k < SSEG; ++k) {
            const T* src = in + L.base + (int64_t)(r0 + k) * L.stride;
            if constexpr (V == 1) v[k] = ld_stream(src);
            else v[k] = *(const vt*)src;
        }
#pragma unroll
        for (int k = 0; k < SSEG; ++k) {
            const T ai = f[M + r0 + k];
            y = v[k] * f[r0 + k] - ai * y;
            mu = -ai * mu;
            v[k] = y;
        }
    }
    const vt yin = segment_carry<vt>(mu, y, seg, nseg, line, lines, false, sh);
    vt x{}, nu = one;
    if (live) {
        T m = T(1);
#pragma unroll
        for (int k = 0; k < SSEG; ++k) {
            m = -f[M + r0 + k] * m;
            v[k] = v[k] + m * yin;
        }
#pragma unroll
        for (int k = SSEG - 1; k >= 0; --k) {
            const T cp = f[2 * M + r0 + k];
            x = v[k] - cp * x;
            nu = -cp * nu;
            v[k] = x;
        }
    }
    const vt xin = segment_carry<vt>(nu, x, seg, nseg, line, lines, true, sh);
    if (live) {
        T n = T(1);
#pragma unroll
        for (int k = SSEG - 1; k >= 0; --k) {
            n = -f[2 * M + r0 + k] * n;
            v[k] = v[k] + n * xin;
        }
#pragma unroll
        for (int k = 0; k < SSEG; ++k) {
            const int64_t idx = L.base + (int64_t)(r0 + k) * L.stride;
            if constexpr (V == 1) {
                sweep_store<T, EPI>(A, idx, v[k]);
            } else if constexpr (EPI == EPI_STORE) {
                *(vt*)((T*)A.out + idx) = v[k];
            } else {
                vt* W = (vt*)((T*)A.out + idx);
                st_stream(W, ld_stream(W) + (T)A.b1 * ld_stream((const vt*)((const T*)A.K1 + idx)) + (T)A.b2 * v[k]);
            }
        }
    }
}

// Lines longer than one block's segments (SEG_BLOCK * seg_rows rows): one block per slot of V
// adjacent lines, walking the line in chunks of SEG_BLOCK * seg_rows rows.  Forward: each chunk runs
// the segmented recurrence with the previous chunk's last d' as the carry into its first segment
// (folded into that segment's affine map, so the block scan gives every segment its true carry) and
// leaves d' in memory (the output, or the consumed input when updating); backward: the chunks in
// reverse, the next chunk's first x as the carry.  sh: 4*SEG_BLOCK + 1 entries of LDS.
template <typename T, int EPI, int V>
__device__ __forceinline__ void sweep_strided_chunked(const DevPlan& P, const SweepArgs& A, const Strided& L, int lm,
                                                      typename lane_vec<T, V>::type* sh)
{
    typedef typename lane_vec<T, V>::type vt;
    const int M = 1 << lm;
    constexpr int SSEG = seg_rows((int)sizeof(T), V);
    constexpr int RB = SEG_BLOCK * SSEG;
    const int nch = M / RB;
    const int seg = threadIdx.x;
    const T* f = (const T*)P.fac + L.fac;
    const T* in = (const T*)A.in;
    T* dst = (EPI == EPI_STORE) ? (T*)A.out : (T*)A.in;
    const vt one = vt{} + T(1);
    vt* cbuf = sh + 4 * SEG_BLOCK;
    vt cin{};
    for (int c = 0; c < nch; ++c) {
        const int r0 = c * RB + seg * SSEG;
        vt v[SSEG];
#pragma unroll
        for (int k = 0; k < SSEG; ++k) {
            const T* src = in + L.base + (int64_t)(r0 + k) * L.stride;
            if constexpr (V == 1) v[k] = ld_stream(src);
            else v[k] = *(const vt*)src;
        }
        vt y{}, mu = one;
#pragma unroll
        for (int k = 0; k < SSEG; ++k) {
            const T ai = f[M + r0 + k];
            y = v[k] * f[r0 + k] - ai * y;
            mu = -ai * mu;
            v[k] = y;
        }
        if (seg == 0) {
            y = y + mu * cin;
            mu = vt{};
        }
        vt yin = segment_carry<vt>(mu, y, seg, SEG_BLOCK, 0, 1, false, sh);
        if (seg == 0) yin = cin;
        T m = T(1);
#pragma unroll
        for (int k = 0; k < SSEG; ++k) {
            m = -f[M + r0 + k] * m;
            v[k] = v[k] + m * yin;
            T* q = dst + L.base + (int64_t)(r0 + k) * L.stride;
            if constexpr (V == 1) *q = v[k];
            else *(vt*)q = v[k];
        }
        if (seg == SEG_BLOCK - 1) cbuf[0] = v[SSEG - 1];
        __syncthreads();
        cin = cbuf[0];
        __syncthreads();
    }
    cin = vt{};
    for (int c = nch - 1; c >= 0; --c) {
        const int r0 = c * RB + seg * SSEG;
        vt v[SSEG];
#pragma unroll
        for (int k = 0; k < SSEG; ++k) {
            const T* src = dst + L.base + (int64_t)(r0 + k) * L.stride;
            if constexpr (V == 1) v[k] = *src;
            else v[k] = *(const vt*)src;
        }
        vt x{}, nu = one;
#pragma unroll
        for (int k = SSEG - 1; k >= 0; --k) {
            const T cp = f[2 * M + r0 + k];
            x = v[k] - cp * x;
            nu = -cp * nu;
            v[k] = x;
        }
        if (seg == SEG_BLOCK - 1) {
            x = x + nu * cin;
            nu = vt{};
        }
        vt xin = segment_carry<vt>(nu, x, seg, SEG_BLOCK, 0, 1, true, sh);
        if (seg == SEG_BLOCK - 1) xin = cin;
        T n = T(1);
#pragma unroll
        for (int k = SSEG - 1; k >= 0; --k) {
            n = -f[2 * M + r0 + k] * n;
            v[k] = v[k] + n * xin;
        }
        if (seg == 0) cbuf[0] = v[0];
#pragma unroll
        for (int k = 0; k < SSEG; ++k) {
            const int64_t idx = L.base + (int64_t)(r0 + k) * L.stride;
            if constexpr (V == 1) {
                sweep_store<T, EPI>(A, idx, v[k]);
            } else if constexpr (EPI == EPI_STORE) {
                *(vt*)((T*)A.out + idx) = v[k];
            } else {
                vt* W = (vt*)((T*)A.out + idx);
                st_stream(W, ld_stream(W) + (T)A.b1 * ld_stream((const vt*)((const T*)A.K1 + idx)) + (T)A.b2 * v[k]);
            }
        }
        __syncthreads();
        cin = cbuf[0];
        __syncthreads();
    }
}

// Strided lines longer than 2^SHORT_LM rows.  Classes up to SEG_BLOCK*seg_rows rows: SEG_BLOCK*seg_rows/M
// line slots of V adjacent lines per block, thread t on slot t mod slots and segment t / slots
// (lanes on consecutive slots, coalesced); longer lines: one block per slot, in chunks.
template <typename T, int EPI, int V>
__global__ __launch_bounds__(SEG_BLOCK) void k_sweep_strided_long(DevPlan P, SweepArgs A, int axis, int64_t blk0)
{
    typedef typename lane_vec<T, V>::type vt;
    __shared__ vt sh[4 * SEG_BLOCK + 1];
    const SweepBlk B = P.ax_blk[axis][blk0 + xcd_block(blockIdx.x, gridDim.x, P.xcd == 2)];
    const int lm = B.lm;
    const int64_t* lo = P.ax_line_off[axis];
    constexpr int SSEG = seg_rows((int)sizeof(T), V);
    if (lm > seg_max_lm((int)sizeof(T), V)) {   // block-uniform branch: one slot of V lines per block
        const int64_t gl = B.line_start;
        int k = B.k_start;
        while (gl >= lo[k + 1]) ++k;
        const UnitDev& U = P.units[P.ax_units[axis][k]];
        sweep_strided_chunked<T, EPI, V>(P, A, strided_geom(P, U, axis, gl - lo[k], lm, A.run), lm, sh);
        return;
    }
    const int slots = (SEG_BLOCK * SSEG) >> lm;
    const int slot = threadIdx.x & (slots - 1);
    const int seg = threadIdx.x >> (__ffs(slots) - 1);
    const int64_t gl = B.line_start + (int64_t)slot * V;
    const bool live = gl < B.line_end;
    Strided L{};
    if (live) {
        int k = B.k_start;
        while (gl >= lo[k + 1]) ++k;
        const UnitDev& U = P.units[P.ax_units[axis][k]];
        L = strided_geom(P, U, axis, gl - lo[k], lm, A.run);
    }
    sweep_strided_seg<T, EPI, V>(P, A, L, lm, live, seg, (1 << lm) / SSEG, slot, slots, sh);
}

// Axis 0 (contiguous lines).  Coefficients are formed on the fly: delta_r = tdiff_0[r] * V^2.
struct Contig {
    int64_t base;
    const void* tdiff;
    double vsq;
    int dir;              // Dirichlet upper face (eq bound1_0): the last row is an identity row
};

template <typename T>
__device__ __forceinline__ Contig contig_geom(const DevPlan& P, const UnitDev& U, int64_t line, int lm)
{
    const int D = P.d;
    int SV = 0;
    for (int k = 0; k < D - 1; ++k) SV += U.lv[k];
    const int64_t loc0 = line << lm;
    const int MV = 1 << U.lv[D - 1];
    const int jv = (int)((loc0 >> SV) & (MV - 1));
    const T* tab = (const T*)P.tab;
    Contig C;
    C.base = U.off + loc0;
    C.tdiff = tab + U.tab[0];
    C.vsq = (double)tab[U.tab[D - 1] + jv];
    C.dir = P.probs[U.prob].dirichlet;
    return C;
}

// Short contiguous line: one thread, Thomas with the line in VGPRs.  g: the line's M values (solved
// in place), td: its tdiff factors, cm = V^2 of the line; dir: the last row sits on a Dirichlet face
// (identity row: zero coupling).
template <typename T, int LM>
__device__ __forceinline__ void reg_solve(T (&g)[1 << LM], const T* td, T cm, T nudt, bool dir)
{
    constexpr int M = 1 << LM;
    T cp[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const T nd = (dir && r == M - 1) ? T(0) : nudt * (td[r] * cm);
        const T b = T(1) + T(2) * nd;
        const T a = (r == 0) ? T(0) : ((r == M - 1) ? -T(2) * nd : -nd);
        const T c = (r == M - 1) ? T(0) : -nd;
        const T inv = T(1) / (r == 0 ? b : b - a * cp[r - 1]);
        cp[r] = c * inv;
        g[r] = (r == 0) ? g[0] * inv : (g[r] - a * g[r - 1]) * inv;
    }
#pragma unroll
    for (int r = M - 2; r >= 0; --r) g[r] = g[r] - cp[r] * g[r + 1];
}

// Wavefront-cooperative transfer of per-lane chunks of CH consecutive elements (CH * sizeof(T) a
// multiple of 16 bytes, chunks 16-byte aligned): the wavefront's 64 chunks move as 16-byte pieces,
// consecutive lanes on consecutive pieces, through the wavefront's LDS tile (rows of CH elements at
// a pitch of CH + one piece), so every global access instruction covers whole cache lines instead of
// one 16-byte piece of 64 different lines.  base: this lane's chunk (element index); ok: the lane
// has a chunk.  Every thread of the block calls these (they contain block barriers).
template <typename T, int CH>
struct ChunkTile {
    static constexpr int VPP = 16 / (int)sizeof(T);   // elements per 16-byte piece
    static constexpr int PPC = CH / VPP;             // pieces per chunk (a power of two)
    static constexpr int PITCH = CH + VPP;           // elements per tile row
    static_assert(CH % VPP == 0, "chunks of whole 16-byte pieces");
};
using piece_t = unsigned int __attribute__((ext_vector_type(4)));

template <typename T, int CH>
__device__ __forceinline__ void chunk_load(const T* g, int64_t base, bool ok, T* tile, T (&x)[CH])
{
    using C = ChunkTile<T, CH>;
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int it = 0; it < C::PPC; ++it) {
        const int q = it * WAVE + lane;
        const int row = q / C::PPC, pc = q % C::PPC;
        const int64_t b = __shfl(base, row);
        const int rok = __shfl(ok ? 1 : 0, row);
        if (rok) *(piece_t*)(tile + row * C::PITCH + pc * C::VPP) = *(const piece_t*)(g + b + pc * C::VPP);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < CH; ++r) x[r] = tile[lane * C::PITCH + r];
}

template <typename T, int CH>
__device__ __forceinline__ void chunk_store(T* g, int64_t base, bool ok, T* tile, const T (&x)[CH])
{
    using C = ChunkTile<T, CH>;
    const int lane = threadIdx.x & (WAVE - 1);
    __syncthreads();                                  // every lane has read its row of the tile
#pragma unroll
    for (int r = 0; r < CH; ++r) tile[lane * C::PITCH + r] = x[r];
    __syncthreads();
#pragma unroll
    for (int it = 0; it < C::PPC; ++it) {
        const int q = it * WAVE + lane;
        const int row = q / C::PPC, pc = q % C::PPC;
        const int64_t b = __shfl(base, row);
        const int rok = __shfl(ok ? 1 : 0, row);
        if (rok) *(piece_t*)(g + b + pc * C::VPP) = *(const piece_t*)(tile + row * C::PITCH + pc * C::VPP);
    }
}

// One thread per short line: the line moves through the tile when it spans whole 16-byte pieces,
// else with plain loads and stores.
template <typename T, int LM>
__device__ __forceinline__ void sweep_contig_reg(const SweepArgs& A, const Contig& L, T nudt, bool ok, T* tile)
{
    constexpr int M = 1 << LM;
    T g[M];
    if constexpr (M * sizeof(T) % 16 == 0) {
        chunk_load<T, M>((const T*)A.in, L.base, ok, tile, g);
        if (ok) reg_solve<T, LM>(g, (const T*)L.tdiff, (T)L.vsq, nudt, L.dir != 0);
        chunk_store<T, M>((T*)A.out, L.base, ok, tile, g);
    } else if (ok) {
        const T* in = (const T*)A.in + L.base;
#pragma unroll
        for (int r = 0; r < M; ++r) g[r] = in[r];
        reg_solve<T, LM>(g, (const T*)L.tdiff, (T)L.vsq, nudt, L.dir != 0);
        T* out = (T*)A.out + L.base;
#pragma unroll
        for (int r = 0; r < M; ++r) out[r] = g[r];
    }
}

// Long contiguous line: SP = M/SEG lanes, each owning SEG consecutive rows.  Each lane eliminates
// its first SEG-1 rows in terms of z_{p-1} (last row of the previous segment) and z_p (its own last
// row): x_k = y_k + v_k z_{p-1} + w_k z_p.  Substituting into the segment-closing rows leaves a
// tridiagonal system in z_0..z_{SP-1}, solved by parallel cyclic reduction across the SP lanes with
// wavefront shuffles; the lanes then reconstruct their rows.  Diagonally dominant: no pivoting.
// g: the lane's SEG rows (contiguous), solved in place; td: their tdiff factors, cm = V^2 of the line.
template <typename T, int SP>
__device__ __forceinline__ void part_solve(T (&g)[SEG], const T* td, T cm, T nudt, int p, bool dir)
{
    constexpr int S = SEG;
    const bool first = (p == 0), last = (p == SP - 1);
    T cp[S - 1], v[S - 1], w[S - 1];
    // interior rows k = 0..S-2 (global r0 + k); row S-1 closes the segment
    T a_first = T(0);
#pragma unroll
    for (int k = 0; k < S - 1; ++k) {
        const T nd = nudt * (td[k] * cm);
        const T b = T(1) + T(2) * nd;
        const T a = (first && k == 0) ? T(0) : -nd;   // interior rows are never the line's last row
        const T c = -nd;
        if (k == 0) {
            a_first = a;
            const T inv = T(1) / b;
            cp[0] = (S - 1 == 1) ? T(0) : c * inv;
            g[0] = g[0] * inv;
            v[0] = -a * inv;
            w[0] = (S - 1 == 1) ? -c * inv : T(0);
        } else {
            const T inv = T(1) / (b - a * cp[k - 1]);
            const bool lastint = (k == S - 2);
            cp[k] = lastint ? T(0) : c * inv;
            g[k] = (g[k] - a * g[k - 1]) * inv;
            v[k] = -a * v[k - 1] * inv;
            w[k] = lastint ? -c * inv : T(0);
        }
    }
#pragma unroll
    for (int k = S - 3; k >= 0; --k) {
        g[k] = g[k] - cp[k] * g[k + 1];
        v[k] = v[k] - cp[k] * v[k + 1];
        w[k] = w[k] - cp[k] * w[k + 1];
    }
    (void)a_first;
    // segment-closing row r0 + S - 1
    const T ndl = (dir && last) ? T(0) : nudt * (td[S - 1] * cm);   // Dirichlet face: identity row
    const T bl = T(1) + T(2) * ndl;
    const T al = last ? -T(2) * ndl : -ndl;
    const T cl = last ? T(0) : -ndl;
    // first interior row of the next segment (y, v, w)
    T yF = __shfl_down(g[0], 1, SP), vF = __shfl_down(v[0], 1, SP), wF = __shfl_down(w[0], 1, SP);
    if (last) yF = vF = wF = T(0);
    T Ar = al * v[S - 2];
    T Br = bl + al * w[S - 2] + cl * vF;
    T Cr = cl * wF;
    T Rr = g[S - 1] - al * g[S - 2] - cl * yF;
    // parallel cyclic reduction over the SP lanes of this line
#pragma unroll
    for (int s = 1; s < SP; s <<= 1) {
        T Am = __shfl_up(Ar, s, SP), Bm = __shfl_up(Br, s, SP), Cm = __shfl_up(Cr, s, SP), Rm = __shfl_up(Rr, s, SP);
        T Ap = __shfl_down(Ar, s, SP), Bp = __shfl_down(Br, s, SP), Cp = __shfl_down(Cr, s, SP), Rp = __shfl_down(Rr, s, SP);
        if (p < s) { Am = T(0); Bm = T(1); Cm = T(0); Rm = T(0); }
        if (p + s >= SP) { Ap = T(0); Bp = T(1); Cp = T(0); Rp = T(0); }
        const T k1 = Ar / Bm, k2 = Cr / Bp;
        const T nA = -k1 * Am, nC = -k2 * Cp;
        const T nB = Br - k1 * Cm - k2 * Ap;
        const T nR = Rr - k1 * Rm - k2 * Rp;
        Ar = nA; Br = nB; Cr = nC; Rr = nR;
    }
    const T z = Rr / Br;
    T zprev = __shfl_up(z, 1, SP);
    if (first) zprev = T(0);
#pragma unroll
    for (int k = 0; k < S - 1; ++k) g[k] = g[k] + v[k] * zprev + w[k] * z;
    g[S - 1] = z;
}

// The lane's SEG rows move through the wavefront's tile in FP32; in FP64 the tile costs more in
// occupancy (the solve holds four SEG-row arrays) than it gains, and the rows are loaded directly.
template <typename T, int SP>
__device__ __forceinline__ void sweep_contig_part(const SweepArgs& A, const Contig& L, T nudt, int p, bool ok, T* tile)
{
    const int r0 = p * SEG;
    T g[SEG];
    if constexpr (sizeof(T) == 4) {
        chunk_load<T, SEG>((const T*)A.in, L.base + r0, ok, tile, g);
        if (ok) part_solve<T, SP>(g, (const T*)L.tdiff + r0, (T)L.vsq, nudt, p, L.dir != 0);   // whole lane groups
        chunk_store<T, SEG>((T*)A.out, L.base + r0, ok, tile, g);
    } else if (ok) {
        const T* in = (const T*)A.in + L.base + r0;
#pragma unroll
        for (int k = 0; k < SEG; ++k) g[k] = in[k];
        part_solve<T, SP>(g, (const T*)L.tdiff + r0, (T)L.vsq, nudt, p, L.dir != 0);
        T* out = (T*)A.out + L.base + r0;
#pragma unroll
        for (int k = 0; k < SEG; ++k) out[k] = g[k];
    }
}

template <typename T, bool LONG>
__global__ __launch_bounds__(LINE_BLOCK) void k_sweep_contig(DevPlan P, SweepArgs A, int64_t blk0)
{
    // one tile per wavefront, sized for chunks of 16 elements (the longest: SEG rows, or a line of
    // 2^CONTIG_REG_LM points)
    static_assert(SEG <= 16 && (1 << CONTIG_REG_LM) <= 16, "chunks fit the tile");
    constexpr int TILE = (LONG && sizeof(T) == 8) ? 1 : WAVE * ChunkTile<T, 16>::PITCH;   // FP64 long: no tile
    __shared__ __align__(16) T tiles[LINE_BLOCK / WAVE][TILE];
    const SweepBlk B = P.ax_blk[0][blk0 + xcd_block(blockIdx.x, gridDim.x, P.xcd == 2)];
    const int lm = B.lm;
    const int sp = lm > CONTIG_REG_LM ? (1 << lm) / SEG : 1;   // lanes per line
    const int64_t gl = B.line_start + threadIdx.x / sp;
    const bool ok = gl < B.line_end;        // lanes past the block's lines stay for the barriers
    const int p = threadIdx.x & (sp - 1);
    Contig L{};
    T nudt = T(0);
    if (ok) {
        const int64_t* lo = P.ax_line_off[0];
        int k = B.k_start;
        while (gl >= lo[k + 1]) ++k;
        const UnitDev& U = P.units[P.ax_units[0][k]];
        L = contig_geom<T>(P, U, gl - lo[k], lm);
        nudt = ((const T*)P.tab)[P.probs[U.prob].cst + CST_RUN + 3 * A.run + 1];
    }
    T* tile = tiles[threadIdx.x / WAVE];
    if constexpr (!LONG) {
        switch (lm) {
        case 0: sweep_contig_reg<T, 0>(A, L, nudt, ok, tile); break;
        case 1: sweep_contig_reg<T, 1>(A, L, nudt, ok, tile); break;
        case 2: sweep_contig_reg<T, 2>(A, L, nudt, ok, tile); break;
        case 3: sweep_contig_reg<T, 3>(A, L, nudt, ok, tile); break;
        case 4: sweep_contig_reg<T, 4>(A, L, nudt, ok, tile); break;
        default: break;
        }
    } else {
        switch (lm) {
        case 5: sweep_contig_part<T, 2>(A, L, nudt, p, ok, tile); break;
        case 6: sweep_contig_part<T, 4>(A, L, nudt, p, ok, tile); break;
        case 7: sweep_contig_part<T, 8>(A, L, nudt, p, ok, tile); break;
        case 8: sweep_contig_part<T, 16>(A, L, nudt, p, ok, tile); break;
        case 9: sweep_contig_part<T, 32>(A, L, nudt, p, ok, tile); break;
        case 10: sweep_contig_part<T, 64>(A, L, nudt, p, ok, tile); break;
        default: break;   // longer lines go to k_sweep_strided_long
        }
    }
}

// ------------------------------------------------------------------------------------------------
// Unit-resident schedule: one workgroup per unit advances it by n AMFR-W steps with W, K1 and two
// work vectors in LDS; W (in and out), F(g) (read per stage) and the tabulated Thomas factors are its
// only global traffic.  A vector holds the axis-1 rows of M_1 nodes at a pitch P = res_pitch(M_1),
// so a node's LDS offset is affine in its indices (strides S_1 = 1, S_2 = P, S_k = P M_2 .. M_{k-1})
// and every neighbour or line element is one add away.  The unit's 1-D coefficient tables follow the
// four vectors.
template <int D>
struct ResGeom {
    int M[D], L[D];   // extents and their log2
    int S[D];         // LDS strides of the axes
    int N[D];         // node-index shifts of the axes (node n = sum_i (j_i - 1) << N_i)
    int tb[D];        // offset of each axis' coefficient table in the LDS table area
    int Pn, P0, MV;
};

// LDS offset of inner node n (0-based node index of the unit).
template <int D>
__device__ __forceinline__ int res_at(const ResGeom<D>& G, int n)
{
    return (n & (G.M[0] - 1)) + (n >> G.L[0]) * G.P0;
}

// Zero-face Sketch-1 operator on LDS vectors, fused with the stage combination OP.  A thread takes
// R consecutive nodes of one axis-1 row (R divides M_1), so every neighbour row is read as a short
// segment at fixed offsets from one address, and the face tests, coefficient products and masks of
// the other axes are formed once for the R nodes.  Lower-face neighbours are 0 and the upper-face
// ghost is the node below the face (eq. bound1); a neighbour beyond a face is read at an index
// inside the unit and replaced by 0 (a 0/1 mask) or by the ghost, and the mixed and advection
// coefficients vanish on the upper faces.
template <typename T, int D, int OP, int R>
__device__ __forceinline__ void res_stencil_r(const ResGeom<D>& G, const T* st, const T* cst, int dirichlet, T sc,
                                              T av, T qv, const T* X0, const T* X1, T* Wout, const T* cGg)
{
    constexpr int NA = D - 1;                     // axes other than axis 1 (0-based 1 .. D-1)
    const T* tv = st + G.tb[D - 1];
    const T* t0 = st + G.tb[0];
    const T tdV = tv[G.MV], tmixV = tv[G.MV + 1];
    const int ng = G.Pn / R;
    auto X = [&](int idx) -> T {
        if constexpr (OP == OP_STAGE2) return X0[idx] + av * X1[idx];
        else return X0[idx];
    };
    for (int g = threadIdx.x; g < ng; g += RES_BLOCK) {
        const int n = g * R;                      // first node of the group
        const int j0 = n & (G.M[0] - 1);
        const bool lo0 = j0 == 0, hi0 = j0 + R == G.M[0];
        int j[D], dm[D], dp[D];
        bool lo[D], hi[D];
        T mk[D];                                  // 0 on the lower face of the axis, else 1
        bool face = false;                        // Dirichlet faces of the rate axes 2..N-1 (axis 1: per node)
#pragma unroll
        for (int i = 1; i < D; ++i) {
            j[i] = (n >> G.N[i]) & (G.M[i] - 1);
            lo[i] = j[i] == 0;
            hi[i] = j[i] == G.M[i] - 1;
            dm[i] = lo[i] ? 0 : G.S[i];
            dp[i] = hi[i] ? 0 : G.S[i];
            mk[i] = lo[i] ? T(0) : T(1);
            if (i < D - 1) face |= dir_face(dirichlet, j[i] + 1, G.M[i]);
        }
        const int at = res_at<D>(G, n);
        // a row segment: positions j0 - 1 .. j0 + R of the row through `base` (the edges clamped to
        // the row: 0 below the lower face, the ghost j0 + R - 2 beyond the upper face)
        auto seg = [&](int base, T (&v)[R + 2]) {
#pragma unroll
            for (int q = 1; q <= R; ++q) v[q] = X(base + q - 1);
            const T l = X(base - (lo0 ? 0 : 1)), h = X(base + R - (hi0 ? 1 : 0));
            v[0] = lo0 ? T(0) : l;
            v[R + 1] = hi0 ? v[R - 1] : h;
        };
        T c[R + 2];
        seg(at, c);
        T acc[R];
        // coefficients of axis 1 per node, of the other axes per group
        T td0[R], tm0[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            td0[q] = t0[j0 + q];
            tm0[q] = t0[G.M[0] + j0 + q];
            acc[q] = td0[q] * (c[q + 2] - T(2) * c[q + 1] + c[q]);
        }
        T tmix[D], tphi[D];
        tmix[0] = T(0);
        tphi[0] = T(0);
#pragma unroll
        for (int i = 1; i < D; ++i) {
            T m[R + 2], p[R + 2];
            seg(at - dm[i], m);
            seg(at + dp[i], p);
#pragma unroll
            for (int q = 0; q < R + 2; ++q) m[q] *= mk[i];          // the row below the lower face is 0
            T tdi;
            if (i < D - 1) {
                const T* ti = st + G.tb[i];
                tdi = ti[j[i]];
                tmix[i] = ti[G.M[i] + j[i]];
                tphi[i] = ti[2 * G.M[i] + j[i]];
            } else {
                tdi = tdV;
                tmix[i] = tmixV;
                tphi[i] = T(0);
            }
            // pair (axis 1, axis i): zero on either upper face
            const T c0i = (i < D - 1) ? cst[CST_RHO + 0 * MAXD + i] : cst[CST_SPHI + 0];
            const T c0t = hi[i] ? T(0) : c0i * tmix[i];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const T xm = m[q + 1];
                const T xp = hi[i] ? xm : p[q + 1];
                acc[q] += tdi * (xp - T(2) * c[q + 1] + xm);
                const bool h0 = hi0 && q == R - 1;
                const T cf = h0 ? T(0) : tm0[q] * c0t;
                acc[q] += cf * (p[q + 2] + m[q] - m[q + 2] - p[q]);
            }
            if (i < D - 1) {                       // advection of the rate axes 2..N-1
                T sacc = T(0);
#pragma unroll
                for (int jj = 1; jj <= i; ++jj) sacc += cst[CST_RHO + i * MAXD + jj] * tphi[jj];
                const T ca = hi[i] ? T(0) : tmix[i] * sacc;
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const T xm = m[q + 1];
                    const T xp = hi[i] ? xm : p[q + 1];
                    acc[q] += ca * (xp - xm);
                }
            }
        }
        // pairs (i, k) of the other axes: corner segments of R nodes
#pragma unroll
        for (int i = 1; i < D - 1; ++i) {
#pragma unroll
            for (int k = i + 1; k < D; ++k) {
                const T cik = (k < D - 1) ? cst[CST_RHO + i * MAXD + k] : cst[CST_SPHI + i];
                const T cf = (hi[i] || hi[k]) ? T(0) : cik * tmix[i] * tmix[k];
                const int bpp = at + dp[i] + dp[k], bmm = at - dm[i] - dm[k];
                const int bpm = at + dp[i] - dm[k], bmp = at - dm[i] + dp[k];
                const T mmm = mk[i] * mk[k];
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const T xx = X(bpp + q) + mmm * X(bmm + q) - mk[k] * X(bpm + q) - mk[i] * X(bmp + q);
                    acc[q] += cf * xx;
                }
            }
        }
        const T vsq = tv[j[D - 1]];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const bool fq = face || dir_face(dirichlet, j0 + q + 1, G.M[0]);
            const T F = fq ? T(0) : vsq * acc[q];
            const int aq = at + q;
            if constexpr (OP == OP_STAGE1) Wout[aq] = sc * (F + cGg[n + q]);
            else if constexpr (OP == OP_STAGE2) Wout[aq] = sc * (F + cGg[n + q]) + qv * X1[aq];
            else Wout[aq] = T(2) * Wout[aq] - c[q + 1] + sc * F;
        }
    }
}

template <typename T, int D, int OP>
__device__ __forceinline__ void res_stencil(const ResGeom<D>& G, const T* st, const T* cst, int dirichlet, T sc,
                                            T av, T qv, const T* X0, const T* X1, T* Wout, const T* cGg)
{
    // two nodes per thread wherever a row allows it, for d <= 4 (four, or two at d >= 5, take so many
    // registers that occupancy halves)
    if (D <= 4 && G.M[0] >= 2) res_stencil_r<T, D, OP, 2>(G, st, cst, dirichlet, sc, av, qv, X0, X1, Wout, cGg);
    else res_stencil_r<T, D, OP, 1>(G, st, cst, dirichlet, sc, av, qv, X0, X1, Wout, cGg);
}

// Solves along one axis of a resident unit (LDS `in` -> LDS `io`, in place when they coincide):
// one thread per line, Thomas with the plan's tabulated factors of the line (inv, a inv, c' of
// (I - nu dt A_ax) for this unit's levels and the line's j_V, as the streaming sweeps use); with
// `upd` the result x updates W += b1 K1 + b2 x instead of being stored.
template <typename T, int D>
__device__ __forceinline__ void res_strided(const ResGeom<D>& G, const T* fa, int ax, const T* in, T* io, bool upd,
                                            T* sW, const T* sK, T b1, T b2)
{
    const int Mi = G.M[ax], Ni = G.N[ax], St = G.S[ax];
    const int lines = G.Pn >> G.L[ax];
    const bool isV = ax == D - 1;
    for (int line = threadIdx.x; line < lines; line += RES_BLOCK) {
        const int lo = line & ((1 << Ni) - 1), hi = line >> Ni;
        const int base = lo + (hi << (Ni + G.L[ax]));          // node index of the line's first row
        const T* f = isV ? fa : fa + (int64_t)((base >> G.N[D - 1]) & (G.MV - 1)) * 3 * Mi;
        int a = res_at<D>(G, base);
        T dprev = T(0);
#pragma unroll 4
        for (int r = 0; r < Mi; ++r, a += St) {
            dprev = in[a] * f[r] - f[Mi + r] * dprev;
            io[a] = dprev;
        }
        a -= St;                                 // row M - 1
        T x = dprev;                             // c'_{M-1} = 0: x_{M-1} = d'_{M-1}
        if (upd) sW[a] = sW[a] + b1 * sK[a] + b2 * x;
#pragma unroll 4
        for (int r = Mi - 2; r >= 0; --r) {
            a -= St;
            x = io[a] - f[2 * Mi + r] * x;
            if (upd) sW[a] = sW[a] + b1 * sK[a] + b2 * x;
            else io[a] = x;
        }
    }
}

// The AMF chain (I - nu dt A_1) .. (I - nu dt A_d) on LDS vectors: axis 0 reads src, the others
// work in place on dst; with upd the last solve ends in W += b1 K1 + b2 K2.
template <typename T, int D>
__device__ __forceinline__ void res_chain(const ResGeom<D>& G, const T* const (&fa)[D], const T* src, T* dst,
                                          bool upd, T* sW, const T* sK, T b1, T b2)
{
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        res_strided<T, D>(G, fa[ax], ax, ax == 0 ? src : dst, dst, upd && ax == D - 1, sW, sK, b1, b2);
        __syncthreads();
    }
}

template <typename T, int D>
__device__ __forceinline__ void resident_unit(const DevPlan& P, const ResArgs& A)
{
    extern __shared__ __align__(16) unsigned char res_smem[];
    const UnitDev U = P.units[blockIdx.x];
    ResGeom<D> G;
    {
        int sh = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            G.L[i] = U.lv[i];
            G.M[i] = 1 << U.lv[i];
            G.N[i] = sh;
            sh += U.lv[i];
        }
        G.Pn = 1 << U.lsum;
        G.MV = G.M[D - 1];
        G.P0 = res_pitch(G.M[0]);
        G.S[0] = 1;
#pragma unroll
        for (int i = 1; i < D; ++i) G.S[i] = (i == 1 ? G.P0 : G.S[i - 1] * G.M[i - 1]);
    }
    const int LP = A.lds_len;
    T* sW = (T*)res_smem;
    T* sK = sW + LP;
    T* sA = sK + LP;
    T* sB = sA + LP;
    T* st = sB + LP;                              // the unit's coefficient tables
    T* Wg = (T*)A.W + U.off;
    const T* cGg = (const T*)A.cG + U.off;
    const T* tab = (const T*)P.tab;
    const T* cst = tab + P.probs[U.prob].cst;
    const int dirp = P.probs[U.prob].dirichlet;
    const T dt = cst[CST_RUN + 3 * A.run], thdt = cst[CST_RUN + 3 * A.run + 2];
    const T a21 = (T)A.a21, q21 = (T)A.q21, b1 = (T)A.b1, b2 = (T)A.b2;
    const T* fac = (const T*)P.fac + (int64_t)A.run * P.fac_run_stride;
    const T* fa[D];
    {
        int at = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int len = i < D - 1 ? 3 * G.M[i] : G.MV + 2;
            const T* src = tab + U.tab[i];
            for (int q = threadIdx.x; q < len; q += RES_BLOCK) st[at + q] = src[q];
            G.tb[i] = at;
            at += len;
            fa[i] = fac + U.fac[i];
        }
    }
    for (int n = threadIdx.x; n < G.Pn; n += RES_BLOCK) sW[res_at<D>(G, n)] = Wg[n];
    __syncthreads();
    for (int s = 0; s < A.nsteps; ++s) {
        // stage 1: K^(0) = dt F(Y); chain; refinement; chain -> K1
        res_stencil<T, D, OP_STAGE1>(G, st, cst, dirp, dt, T(0), T(0), sW, nullptr, sA, cGg);
        __syncthreads();
        res_chain<T, D>(G, fa, sA, sB, false, sW, sK, b1, b2);
        res_stencil<T, D, OP_REFINE>(G, st, cst, dirp, thdt, T(0), T(0), sB, nullptr, sA, cGg);
        __syncthreads();
        res_chain<T, D>(G, fa, sA, sK, false, sW, sK, b1, b2);
        // stage 2: K^(0) = dt F(Y + a21 K1) + q21 K1; chain; refinement; chain ending in the update
        res_stencil<T, D, OP_STAGE2>(G, st, cst, dirp, dt, a21, q21, sW, sK, sA, cGg);
        __syncthreads();
        res_chain<T, D>(G, fa, sA, sB, false, sW, sK, b1, b2);
        res_stencil<T, D, OP_REFINE>(G, st, cst, dirp, thdt, T(0), T(0), sB, nullptr, sA, cGg);
        __syncthreads();
        res_chain<T, D>(G, fa, sA, sB, true, sW, sK, b1, b2);
    }
    for (int n = threadIdx.x; n < G.Pn; n += RES_BLOCK) Wg[n] = sW[res_at<D>(G, n)];
}

template <typename T, int D>
__global__ __launch_bounds__(RES_BLOCK) void k_resident(DevPlan P, ResArgs A)
{
    resident_unit<T, D>(P, A);
}

// The same kernel held to 128 registers (four wavefronts per SIMD): FP32 with d <= 4 spills a few
// registers and runs faster at the higher occupancy; larger d and FP64 would spill far more.
template <typename T, int D>
__global__ __launch_bounds__(RES_BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_resident_w4(DevPlan P, ResArgs A)
{
    resident_unit<T, D>(P, A);
}

template <typename T>
__global__ void k_unit_values(DevPlan P, const T* W, double* vals)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= P.n_units) return;
    const UnitDev U = P.units[u];
    const ProbDev& PR = P.probs[U.prob];
    const int D = P.d;
    int c[MAXD];
    double t[MAXD], h[MAXD];
    for (int i = 0; i < D; ++i) {
        const int M = 1 << U.lv[i];
        h[i] = PR.xmax[i] / (double)M;
        int cc = (int)floor(PR.xeval[i] / h[i]);
        cc = cc > M - 1 ? M - 1 : (cc < 0 ? 0 : cc);
        c[i] = cc;
        t[i] = (PR.xeval[i] - (double)cc * h[i]) / h[i];
    }
    double v = 0.0;
    for (int corner = 0; corner < (1 << D); ++corner) {
        double wgt = 1.0;
        bool onface = false;
        int64_t off = 0;
        int sh = 0;
        double x[MAXD];
        for (int i = 0; i < D; ++i) {
            const int upb = (corner >> i) & 1;
            wgt *= upb ? t[i] : 1.0 - t[i];
            const int jc = c[i] + upb;
            x[i] = (double)jc * h[i];
            if (jc == 0) onface = true;
            else off += (int64_t)(jc - 1) << sh;
            sh += U.lv[i];
        }
        const double val = (onface ? 0.0 : (double)W[U.off + off]) + payoff_at(PR, D - 1, x);
        v += wgt * val;
    }
    vals[u] = v;
}

// Per problem: discount * sum_l c_l u_l in unit order (FP64); Richardson (8 P_fine - P_coarse) / 7
// when coarse values are given.
__global__ void k_combine(DevPlan P, const double* coef, const double* vals, const double* coarse,
                          double* prices)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n_probs) return;
    const ProbDev& PR = P.probs[p];
    double s = 0.0, sc = 0.0;
    for (int u = PR.unit_begin; u < PR.unit_end; ++u) {
        s += coef[u] * vals[u];
        if (coarse) sc += coef[u] * coarse[u];
    }
    double price = PR.discount * s;
    if (coarse) price = (8.0 * price - PR.discount * sc) / 7.0;
    prices[p] = price;
}

// ------------------------------------------------------------------------------------------------
// Stage combinations of schemes with more than two stages: out = (acc ? out : 0) + sum_j c_j in_j
// over every element (padding included, which stays 0).  Four elements per thread.
template <typename T>
__global__ __launch_bounds__(NODE_BLOCK) void k_lincomb(int64_t total, LinArgs A)
{
    const int64_t g0 = ((int64_t)blockIdx.x * NODE_BLOCK + threadIdx.x) * 4;
    if (g0 >= total) return;                  // total is a multiple of UNIT_ALIGN (>= 4)
    T v[4];
    T* out = (T*)A.out;
    if (A.acc) load_vec<T, 4>(out + g0, v);
    else {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = T(0);
    }
#pragma unroll
    for (int j = 0; j < LIN_MAX; ++j) {
        if (j < A.n) {
            T w[4];
            load_vec<T, 4>((const T*)A.in[j] + g0, w);
            const T c = (T)A.c[j];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] += c * w[r];
        }
    }
    store_vec<T, 4>(out + g0, v);
}

// ------------------------------------------------------------------------------------------------
// (I - theta dt P) x = rhs, P the lower triangle (diagonal included) of the Sketch-1 matrix in the
// theta_0 order (Section 4.2, eq (GS)), on every unit.  Row J reads x at its lower neighbours: J - E_0
// on its own axis-0 line, and J - E_k, J - E_i - E_k, J + E_i - E_k (i < k, k >= 1) on axis-0 lines
// whose index r = (j_1, .., j_{d-1}) has a smaller h(r) = sum_{i>=1} i (j_i - 1).  The lines of one
// hyperplane h = const are therefore independent: one workgroup per unit walks the hyperplanes in
// order with a barrier between them (the host lists each unit's lines by hyperplane).  Along a line
// the row recurrence x_j = alpha_j + beta_j x_{j-1} is split into `lanes` segments of ROWS rows,
// segments on consecutive lanes of one wave, joined by a shuffle scan of their affine maps.
// Neighbours on a lower face are 0 (stage increments); Dirichlet rate faces (eq bound1_0) are 0.
template <typename T, int D, int ROWS>
__device__ __forceinline__ void lower_segment(const DevPlan& P, const UnitDev& U, const ProbDev& PR,
                                              const T* tab, const T* cst, T thdt, const T* rhs, T* x,
                                              int64_t line, bool live, int pos, int lanes)
{
    T al[ROWS], be[ROWS];
    int M[D], Sh[D], j[D];
    {
        int sh = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            M[i] = 1 << U.lv[i];
            Sh[i] = sh;
            sh += U.lv[i];
        }
    }
    const int64_t lbase = live ? (line << U.lv[0]) : 0;     // loc of the line's first row
#pragma unroll
    for (int i = 1; i < D; ++i) j[i] = (int)((lbase >> Sh[i]) & (M[i] - 1)) + 1;
    const T* tV = tab + U.tab[D - 1];
    const int MV = M[D - 1];
    const T vsq = tV[j[D - 1] - 1];
    // per-line factors of the axes 1..d-1 (the line's j_1..j_{d-1} are fixed)
    T tdiff[D], tmix[D], tphi[D];
    tdiff[D - 1] = tV[MV];
    tmix[D - 1] = tV[MV + 1];
    tphi[D - 1] = T(0);
#pragma unroll
    for (int i = 1; i < D - 1; ++i) {
        const T* ti = tab + U.tab[i];
        tdiff[i] = ti[j[i] - 1];
        tmix[i] = ti[M[i] + j[i] - 1];
        tphi[i] = ti[2 * M[i] + j[i] - 1];
    }
    bool rowface = false;
#pragma unroll
    for (int i = 1; i < D - 1; ++i) rowface |= dir_face(PR.dirichlet, j[i], M[i]);
    const T* t0 = tab + U.tab[0];
    T y = T(0), mu = T(1);
    if (live) {
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const int j0 = pos * ROWS + k + 1;
            const int64_t J = lbase + (j0 - 1);
            tdiff[0] = t0[j0 - 1];
            tmix[0] = t0[M[0] + j0 - 1];
            T sd = T(0);
#pragma unroll
            for (int i = 0; i < D; ++i) sd += tdiff[i];
            const T diag = T(1) + thdt * vsq * (T(2) * sd);
            T known = T(0);
            // J - E_k, k >= 1: second difference (doubled by the Neumann ghost at j_k = M_k) and the
            // advection of paper axes 2..N-1 (none on the upper face)
#pragma unroll
            for (int k1 = 1; k1 < D; ++k1) {
                if (j[k1] > 1) {
                    T c = tdiff[k1] * (j[k1] == M[k1] ? T(2) : T(1));
                    if (k1 < D - 1 && j[k1] != M[k1]) {
                        T sa = T(0);
#pragma unroll
                        for (int jj = 1; jj <= k1; ++jj) sa += cst[CST_RHO + k1 * MAXD + jj] * tphi[jj];
                        c -= tmix[k1] * sa;
                    }
                    known += c * x[J - ((int64_t)1 << Sh[k1])];
                }
            }
            // mixed pairs (i, k), i < k: J - E_i - E_k (+) and J + E_i - E_k (-), none on an upper face
#pragma unroll
            for (int i = 0; i < D - 1; ++i) {
#pragma unroll
                for (int k1 = i + 1; k1 < D; ++k1) {
                    const int ji = i == 0 ? j0 : j[i];
                    if (ji == M[i] || j[k1] == M[k1] || j[k1] == 1) continue;
                    const T cik = ((k1 < D - 1) ? cst[CST_RHO + i * MAXD + k1] : cst[CST_SPHI + i]) *
                                  tmix[i] * tmix[k1];
                    const int64_t Ei = (int64_t)1 << Sh[i], Ek = (int64_t)1 << Sh[k1];
                    T v = -x[J + Ei - Ek];
                    if (ji > 1) v += x[J - Ei - Ek];
                    known += cik * v;
                }
            }
            const bool face = rowface || dir_face(PR.dirichlet, j0, M[0]);
            const T a = face ? T(0) : (rhs[J] + thdt * vsq * known) / diag;
            const T b = (face || j0 == 1) ? T(0)
                                          : thdt * vsq * tdiff[0] * (j0 == M[0] ? T(2) : T(1)) / diag;
            al[k] = a;
            be[k] = b;
            y = a + b * y;
            mu = b * mu;
        }
    }
    // carry entering the segment: the value of x at the row before it (0 before the line)
    const T xin = wave_carry<T>(mu, y, pos, lanes, false);
    if (live) {
        T xv = xin;
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            xv = al[k] + be[k] * xv;
            x[lbase + pos * ROWS + k] = xv;
        }
    }
}

template <typename T, int D, int ROWS>
__device__ __forceinline__ void lower_unit(const DevPlan& P, const UnitDev& U, int u, const LowerArgs& A)
{
    const ProbDev& PR = P.probs[U.prob];
    const T* tab = (const T*)P.tab;
    const T* cst = tab + PR.cst;
    const T thdt = cst[CST_RUN + 3 * A.run + 2];
    const T* rhs = (const T*)A.rhs + U.off;
    T* x = (T*)A.x + U.off;
    const int M0 = 1 << U.lv[0];
    const int lanes = M0 / ROWS;                        // segments per line (<= 64)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per_wave = 64 / lanes;
    const int slots = per_wave * (LOWER_BLOCK / 64);
    const int slot = wave * per_wave + lane / lanes;
    const int pos = lane % lanes;
    for (int p = P.gs_unit_plane0[u]; p < P.gs_unit_plane0[u + 1]; ++p) {
        const int64_t l0 = P.gs_plane_line0[p], l1 = P.gs_plane_line0[p + 1];
        for (int64_t b = l0; b < l1; b += slots) {      // block-uniform trip count
            const int64_t k = b + slot;
            const bool live = k < l1;
            const int64_t line = live ? P.gs_lines[k] : 0;
            lower_segment<T, D, ROWS>(P, U, PR, tab, cst, thdt, rhs, x, line, live, pos, lanes);
        }
        __syncthreads();                                // the plane's rows before the next plane's
    }
}

template <typename T, int D>
__global__ __launch_bounds__(LOWER_BLOCK) void k_lower(DevPlan P, LowerArgs A)
{
    const int u = blockIdx.x;
    const UnitDev U = P.units[u];
    // rows per lane: lines up to 64 rows take one lane per row, longer ones 64 lanes (<= 16 rows each)
    switch (U.lv[0] <= 6 ? 0 : U.lv[0] - 6) {          // block-uniform
    case 0: lower_unit<T, D, 1>(P, U, u, A); break;
    case 1: lower_unit<T, D, 2>(P, U, u, A); break;
    case 2: lower_unit<T, D, 4>(P, U, u, A); break;
    case 3: lower_unit<T, D, 8>(P, U, u, A); break;
    default: lower_unit<T, D, 16>(P, U, u, A); break;  // axis-1 levels above CONTIG_PART_LM are rejected
    }
}

// ------------------------------------------------------------------------------------------------
// Launchers

template <typename T, int MODE>
static hipError_t node_t(const DevPlan& P, const void* W, void* Y, hipStream_t s)
{
    dim3 g((unsigned)P.n_node_blocks), b(NODE_BLOCK);
    switch (P.d) {
    case 2: hipLaunchKernelGGL((k_node<T, 2, MODE>), g, b, 0, s, P, (const T*)W, (T*)Y); break;
    case 3: hipLaunchKernelGGL((k_node<T, 3, MODE>), g, b, 0, s, P, (const T*)W, (T*)Y); break;
    case 4: hipLaunchKernelGGL((k_node<T, 4, MODE>), g, b, 0, s, P, (const T*)W, (T*)Y); break;
    case 5: hipLaunchKernelGGL((k_node<T, 5, MODE>), g, b, 0, s, P, (const T*)W, (T*)Y); break;
    case 6: hipLaunchKernelGGL((k_node<T, 6, MODE>), g, b, 0, s, P, (const T*)W, (T*)Y); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_payoff(const DevPlan& P, int prec, void* Y, hipStream_t s)
{
    if (P.total == 0) return hipSuccess;
    return prec == 0 ? node_t<double, 0>(P, nullptr, Y, s) : node_t<float, 0>(P, nullptr, Y, s);
}

hipError_t launch_fill_zero(const DevPlan& P, int prec, void* Y, hipStream_t s)
{
    if (P.total == 0) return hipSuccess;
    return prec == 0 ? node_t<double, 1>(P, nullptr, Y, s) : node_t<float, 1>(P, nullptr, Y, s);
}

hipError_t launch_state_read(const DevPlan& P, int prec, const void* W, void* Y, hipStream_t s)
{
    if (P.total == 0) return hipSuccess;
    return prec == 0 ? node_t<double, 2>(P, W, Y, s) : node_t<float, 2>(P, W, Y, s);
}

// One launch of the unfused operator over the block list `list` at R nodes per thread.
template <typename T, int D, int R>
static void stencil_vec_list(const DevPlan& P, int op, const StencilArgs& a, int list, hipStream_t s)
{
    if (P.vblk_n[list] <= 0) return;
    dim3 g((unsigned)P.vblk_n[list]), b(NODE_BLOCK);
    switch (op) {
    case OP_STAGE1: hipLaunchKernelGGL((k_stencil_vec<T, D, OP_STAGE1, R, false>), g, b, 0, s, P, a, list); break;
    case OP_STAGE2: hipLaunchKernelGGL((k_stencil_vec<T, D, OP_STAGE2, R, false>), g, b, 0, s, P, a, list); break;
    default: hipLaunchKernelGGL((k_stencil_vec<T, D, OP_REFINE, R, false>), g, b, 0, s, P, a, list); break;
    }
}

// The streaming operator at up to R consecutive axis-1 nodes per thread.  Fused: one launch, R for
// every unit.  Unfused: every unit at min(R, M_1), one launch per axis-1 line class present.
template <typename T, int D, int R>
static hipError_t stencil_vec(const DevPlan& P, int op, const StencilArgs& a, hipStream_t s)
{
    if (op != OP_STAGE1 && op != OP_STAGE2 && op != OP_REFINE) return hipErrorInvalidValue;
    if (a.S != nullptr) {
        dim3 g((unsigned)P.n_blocks_r[r_index(R)]), b(NODE_BLOCK);
        switch (op) {
        case OP_STAGE1: hipLaunchKernelGGL((k_stencil_vec<T, D, OP_STAGE1, R, true>), g, b, 0, s, P, a, 0); break;
        case OP_STAGE2: hipLaunchKernelGGL((k_stencil_vec<T, D, OP_STAGE2, R, true>), g, b, 0, s, P, a, 0); break;
        default: hipLaunchKernelGGL((k_stencil_vec<T, D, OP_REFINE, R, true>), g, b, 0, s, P, a, 0); break;
        }
        return hipGetLastError();
    }
    if constexpr (R > 1) stencil_vec_list<T, D, 1>(P, op, a, vb_exact(1), s);
    if constexpr (R > 2) stencil_vec_list<T, D, 2>(P, op, a, vb_exact(2), s);
    if constexpr (R > 4) stencil_vec_list<T, D, 4>(P, op, a, vb_exact(4), s);
    stencil_vec_list<T, D, R>(P, op, a, vb_atleast(R), s);
    return hipGetLastError();
}

template <typename T, int D>
static hipError_t march_td(const DevPlan& P, int op, const StencilArgs& a, hipStream_t s)
{
    if constexpr (D > 4) {
        return hipErrorInvalidValue;
    } else {
        dim3 g((unsigned)(P.xcd ? P.n_march_x : P.n_march)), b(MARCH_THREADS);
        const size_t shm = (size_t)P.march_lds;
        switch (op) {
        case OP_STAGE1: hipLaunchKernelGGL((k_march<T, D, OP_STAGE1>), g, b, shm, s, P, a); break;
        case OP_STAGE2: hipLaunchKernelGGL((k_march<T, D, OP_STAGE2>), g, b, shm, s, P, a); break;
        case OP_REFINE: hipLaunchKernelGGL((k_march<T, D, OP_REFINE>), g, b, shm, s, P, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
}

template <typename T, int D>
static hipError_t stencil_td(const DevPlan& P, int op, const StencilArgs& a, hipStream_t s)
{
    const bool hot = op == OP_STAGE1 || op == OP_STAGE2 || op == OP_REFINE;
    // the marching operator solves (with a.S) the axis-1 lines of the grids whose lines fit a tile row
    if (hot && P.march && P.n_march > 0) return march_td<T, D>(P, op, a, s);
    if (hot && P.stencil_r == 8) return stencil_vec<T, D, 8>(P, op, a, s);
    if (hot && P.stencil_r == 4) return stencil_vec<T, D, 4>(P, op, a, s);
    if (hot && P.stencil_r == 2) return stencil_vec<T, D, 2>(P, op, a, s);
    if (a.S != nullptr) return hipErrorInvalidValue;     // the fused form needs 2 or 4 nodes per thread
    dim3 g((unsigned)P.n_node_blocks), b(NODE_BLOCK);
    switch (op) {
    case OP_F_PAYOFF: hipLaunchKernelGGL((k_stencil<T, D, OP_F_PAYOFF>), g, b, 0, s, P, a); break;
    case OP_F_ZERO: hipLaunchKernelGGL((k_stencil<T, D, OP_F_ZERO>), g, b, 0, s, P, a); break;
    case OP_STAGE1: hipLaunchKernelGGL((k_stencil<T, D, OP_STAGE1>), g, b, 0, s, P, a); break;
    case OP_STAGE2: hipLaunchKernelGGL((k_stencil<T, D, OP_STAGE2>), g, b, 0, s, P, a); break;
    case OP_REFINE: hipLaunchKernelGGL((k_stencil<T, D, OP_REFINE>), g, b, 0, s, P, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t stencil_t(const DevPlan& P, int op, const StencilArgs& a, hipStream_t s)
{
    switch (P.d) {
    case 2: return stencil_td<T, 2>(P, op, a, s);
    case 3: return stencil_td<T, 3>(P, op, a, s);
    case 4: return stencil_td<T, 4>(P, op, a, s);
    case 5: return stencil_td<T, 5>(P, op, a, s);
    case 6: return stencil_td<T, 6>(P, op, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stencil(const DevPlan& P, int prec, int op, const StencilArgs& a, hipStream_t s)
{
    if (P.total == 0) return hipSuccess;
    return prec == 0 ? stencil_t<double>(P, op, a, s) : stencil_t<float>(P, op, a, s);
}

template <typename T, bool LONG>
static void sweep_part(const DevPlan& P, int axis, int epi, const SweepArgs& a, int64_t b0, int64_t nb,
                       hipStream_t s)
{
    dim3 g((unsigned)nb), b(LINE_BLOCK), bl(SEG_BLOCK);
    if (axis == 0 && LONG) {
        // lines up to 2^CONTIG_PART_LM: lanes of one wavefront; longer: the segmented block solver
        const int64_t n1 = std::min<int64_t>(nb, std::max<int64_t>(0, P.ax0_nblk_part - b0));
        if (n1 > 0) hipLaunchKernelGGL((k_sweep_contig<T, true>), dim3((unsigned)n1), b, 0, s, P, a, b0);
        if (nb > n1)
            hipLaunchKernelGGL((k_sweep_strided_long<T, EPI_STORE, 1>), dim3((unsigned)(nb - n1)), bl, 0, s, P, a, 0,
                               b0 + n1);
    } else if (axis == 0) hipLaunchKernelGGL((k_sweep_contig<T, LONG>), g, b, 0, s, P, a, b0);
    else if (!LONG && epi == EPI_STORE) hipLaunchKernelGGL((k_sweep_strided<T, EPI_STORE>), g, b, 0, s, P, a, axis, b0);
    else if (!LONG) hipLaunchKernelGGL((k_sweep_strided<T, EPI_UPDATE>), g, b, 0, s, P, a, axis, b0);
    else {
        constexpr int VW = 16 / (int)sizeof(T);
        const bool vec = P.ax_vec[axis] > 1;
        if (epi == EPI_STORE) {
            if (vec) hipLaunchKernelGGL((k_sweep_strided_long<T, EPI_STORE, VW>), g, bl, 0, s, P, a, axis, b0);
            else hipLaunchKernelGGL((k_sweep_strided_long<T, EPI_STORE, 1>), g, bl, 0, s, P, a, axis, b0);
        } else {
            if (vec) hipLaunchKernelGGL((k_sweep_strided_long<T, EPI_UPDATE, VW>), g, bl, 0, s, P, a, axis, b0);
            else hipLaunchKernelGGL((k_sweep_strided_long<T, EPI_UPDATE, 1>), g, bl, 0, s, P, a, axis, b0);
        }
    }
}

hipError_t launch_sweep(const DevPlan& P, int prec, int axis, int epi, int part, const SweepArgs& a,
                        hipStream_t s)
{
    // the update form runs on the last axis only (its short-line blocks hold one slot per thread)
    if (epi != EPI_STORE && axis != P.d - 1) return hipErrorInvalidValue;
    const int64_t ns = P.ax_nblk_short[axis];
    const int64_t b0 = part == 0 ? 0 : ns;
    const int64_t nb = part == 0 ? ns : P.ax_nblk[axis] - ns;
    if (nb <= 0) return hipSuccess;
    if (prec == 0) {
        if (part == 0) sweep_part<double, false>(P, axis, epi, a, b0, nb, s);
        else sweep_part<double, true>(P, axis, epi, a, b0, nb, s);
    } else {
        if (part == 0) sweep_part<float, false>(P, axis, epi, a, b0, nb, s);
        else sweep_part<float, true>(P, axis, epi, a, b0, nb, s);
    }
    return hipGetLastError();
}

// Index of the first non-finite price (-1 if none): one block, min-reduction in LDS.
__global__ __launch_bounds__(256) void k_first_nonfinite(const double* p, int n, int32_t* flag)
{
    __shared__ int best[256];
    int m = INT32_MAX;
    for (int i = threadIdx.x; i < n; i += 256)
        if (!isfinite(p[i]) && i < m) m = i;
    best[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) best[threadIdx.x] = min(best[threadIdx.x], best[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) flag[0] = best[0] == INT32_MAX ? -1 : best[0];
}

__global__ void k_scatter(const double* src, const int32_t* idx, int n, double* dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[idx[i]] = src[i];
}

hipError_t launch_first_nonfinite(const double* p, int n, int32_t* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_first_nonfinite, dim3(1), dim3(256), 0, s, p, n, flag);
    return hipGetLastError();
}

hipError_t launch_scatter(const double* src, const int32_t* idx, int n, double* dst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3((n + 255) / 256), dim3(256), 0, s, src, idx, n, dst);
    return hipGetLastError();
}

template <typename T>
static hipError_t lincomb_t(const DevPlan& P, const LinArgs& a, hipStream_t s)
{
    const int64_t nb = (P.total / 4 + NODE_BLOCK - 1) / NODE_BLOCK;
    hipLaunchKernelGGL((k_lincomb<T>), dim3((unsigned)nb), dim3(NODE_BLOCK), 0, s, P.total, a);
    return hipGetLastError();
}

hipError_t launch_lincomb(const DevPlan& P, int prec, const LinArgs& a, hipStream_t s)
{
    if (P.total == 0) return hipSuccess;
    if (a.n < 0 || a.n > LIN_MAX || (P.total & 3)) return hipErrorInvalidValue;
    return prec == 0 ? lincomb_t<double>(P, a, s) : lincomb_t<float>(P, a, s);
}

template <typename T>
static hipError_t lower_t(const DevPlan& P, const LowerArgs& a, hipStream_t s)
{
    dim3 g((unsigned)P.n_units), b(LOWER_BLOCK);
    switch (P.d) {
    case 2: hipLaunchKernelGGL((k_lower<T, 2>), g, b, 0, s, P, a); break;
    case 3: hipLaunchKernelGGL((k_lower<T, 3>), g, b, 0, s, P, a); break;
    case 4: hipLaunchKernelGGL((k_lower<T, 4>), g, b, 0, s, P, a); break;
    case 5: hipLaunchKernelGGL((k_lower<T, 5>), g, b, 0, s, P, a); break;
    case 6: hipLaunchKernelGGL((k_lower<T, 6>), g, b, 0, s, P, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lower(const DevPlan& P, int prec, const LowerArgs& a, hipStream_t s)
{
    if (P.n_units == 0) return hipSuccess;
    if (!P.gs_unit_plane0 || !P.gs_plane_line0 || !P.gs_lines) return hipErrorInvalidValue;
    return prec == 0 ? lower_t<double>(P, a, s) : lower_t<float>(P, a, s);
}

template <typename T>
static hipError_t resident_t(const DevPlan& P, const ResArgs& a, hipStream_t s)
{
    dim3 g((unsigned)P.n_units), b(RES_BLOCK);
    const size_t shm = ((size_t)4 * a.lds_len + (size_t)a.tab_len) * sizeof(T);
    switch (P.d) {
    case 2: hipLaunchKernelGGL((k_resident<T, 2>), g, b, shm, s, P, a); break;
    case 3:
        if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((k_resident_w4<T, 3>), g, b, shm, s, P, a);
        else hipLaunchKernelGGL((k_resident<T, 3>), g, b, shm, s, P, a);
        break;
    case 4:
        if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((k_resident_w4<T, 4>), g, b, shm, s, P, a);
        else hipLaunchKernelGGL((k_resident<T, 4>), g, b, shm, s, P, a);
        break;
    case 5: hipLaunchKernelGGL((k_resident<T, 5>), g, b, shm, s, P, a); break;
    case 6: hipLaunchKernelGGL((k_resident<T, 6>), g, b, shm, s, P, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_resident(const DevPlan& P, int prec, const ResArgs& a, hipStream_t s)
{
    if (P.n_units == 0 || a.nsteps <= 0) return hipSuccess;
    return prec == 0 ? resident_t<double>(P, a, s) : resident_t<float>(P, a, s);
}

hipError_t launch_unit_values(const DevPlan& P, int prec, const void* W, double* vals, hipStream_t s)
{
    if (P.n_units == 0) return hipSuccess;
    dim3 g((P.n_units + 127) / 128), b(128);
    if (prec == 0) hipLaunchKernelGGL((k_unit_values<double>), g, b, 0, s, P, (const double*)W, vals);
    else hipLaunchKernelGGL((k_unit_values<float>), g, b, 0, s, P, (const float*)W, vals);
    return hipGetLastError();
}

hipError_t launch_combine(const DevPlan& P, const double* coef, const double* vals,
                          const double* coarse, double* prices, hipStream_t s)
{
    if (P.n_probs == 0) return hipSuccess;
    dim3 g((P.n_probs + 63) / 64), b(64);
    hipLaunchKernelGGL(k_combine, g, b, 0, s, P, coef, vals, coarse, prices);
    return hipGetLastError();
}

}  // namespace amf
