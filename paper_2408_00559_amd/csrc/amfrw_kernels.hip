// gfx950 kernels of libamfrw: payoff initialisation, the explicit operator of Sketch 1 fused with
// the AMFR-W stage combinations, the directional tridiagonal solves of Lemma lema:ls, tensor-product
// interpolation and the FP64 combination of component-grid values.
//
// Layout: every grid vector stores the inner nodes of all units back to back; inside a unit axis 0
// is fastest and M_i = 2^lv_i, so index decoding is shifts and masks.  Lower-face (Outer) values are
// never stored: they are the payoff for solution vectors and 0 for increments.
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

__device__ __forceinline__ int find_unit(const UnitDev* units, int u, int64_t g)
{
    while (g >= units[u + 1].off) ++u;
    return u;
}

// ------------------------------------------------------------------------------------------------
// Initial data (dis0): Y = g at every inner node.
template <typename T, int D>
__global__ __launch_bounds__(NODE_BLOCK) void k_init(DevPlan P, T* Y)
{
    const int64_t g = (int64_t)blockIdx.x * NODE_BLOCK + threadIdx.x;
    if (g >= P.total) return;
    const int u = find_unit(P.units, P.blk_unit[blockIdx.x], g);
    const UnitDev U = P.units[u];
    const ProbDev& PR = P.probs[U.prob];
    const int64_t loc = g - U.off;
    double x[MAXD];
    int sh = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const int M = 1 << U.lv[i];
        const int j = (int)((loc >> sh) & (M - 1)) + 1;
        x[i] = (double)j * (PR.xmax[i] / (double)M);
        sh += U.lv[i];
    }
    Y[g] = (T)payoff_at(PR, D - 1, x);
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
    const int64_t g = (int64_t)blockIdx.x * NODE_BLOCK + threadIdx.x;
    if (g >= P.total) return;
    const int u = find_unit(P.units, P.blk_unit[blockIdx.x], g);
    const UnitDev U = P.units[u];
    const ProbDev& PR = P.probs[U.prob];
    const T* tab = (const T*)P.tab;
    const T* cst = tab + PR.cst;
    const int64_t loc = g - U.off;

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
        if constexpr (OP == OP_STAGE) return X0[idx] + av * X1[idx];
        else return X0[idx];
    };
    constexpr bool payface = (OP == OP_F_PAYOFF || OP == OP_STAGE);
    // value at j + si e_i + sk e_k when that node lies on a lower face
    auto face = [&](int i, int si, int k, int sk) -> T {
        if constexpr (!payface) {
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
    const T F = vsq * acc;
    const T sc = A.scale_sel < 0 ? (T)A.scale : cst[A.scale_sel];
    T* W = (T*)A.W;
    if constexpr (OP == OP_F_PAYOFF || OP == OP_F_ZERO) {
        W[g] = sc * F;
    } else if constexpr (OP == OP_STAGE) {
        W[g] = sc * F + (T)A.q * X1[g];
    } else {
        W[g] = T(2) * W[g] - X0[g] + sc * F;
    }
}

// ------------------------------------------------------------------------------------------------
// Directional solve (I - nu dt A_i) x = G along one line (Lemma lema:ls): rows r = 0..M-1 with
// delta_r = d_i / h_i^2, diagonal 1 + 2 nu dt delta_r, super-diagonal -nu dt delta_r (none in the
// last row), sub-diagonal -nu dt delta_r (none in the first row, doubled in the last row: Neumann).
struct LineGeom {
    int64_t base;     // element index of row 0
    int64_t stride;   // E_axis
    const void* dtab; // rate axis: tdiff block; V axis: vsq block
    double cmul;      // rate axis: vsq(j_V); V axis: tdiff_V
};

template <typename T>
__device__ __forceinline__ LineGeom line_geom(const DevPlan& P, const UnitDev& U, int axis,
                                              int64_t line, int lm)
{
    const int D = P.d;
    int S = 0, SV = 0;
    for (int k = 0; k < axis; ++k) S += U.lv[k];
    for (int k = 0; k < D - 1; ++k) SV += U.lv[k];
    const int64_t E = (int64_t)1 << S;
    const int64_t lo = line & (E - 1), hi = line >> S;
    const int64_t loc0 = lo + (hi << (S + lm));
    const T* tab = (const T*)P.tab;
    const T* tV = tab + U.tab[D - 1];
    const int MV = 1 << U.lv[D - 1];
    LineGeom L;
    L.base = U.off + loc0;
    L.stride = E;
    if (axis < D - 1) {
        const int jV = (int)((loc0 >> SV) & (MV - 1)) + 1;
        L.dtab = tab + U.tab[axis];
        L.cmul = (double)tV[jV - 1];
    } else {
        L.dtab = tV;
        L.cmul = (double)tV[MV];
    }
    return L;
}

template <typename T, int EPI>
__device__ __forceinline__ void sweep_store(const SweepArgs& A, int64_t idx, T x)
{
    if constexpr (EPI == EPI_STORE) {
        ((T*)A.out)[idx] = x;
    } else {
        T* Y = (T*)A.out;
        Y[idx] = Y[idx] + (T)A.b1 * ((const T*)A.K1)[idx] + (T)A.b2 * x;
    }
}

// Short lines: Thomas with the whole line's factors in registers.
template <typename T, int LM, int EPI>
__device__ __forceinline__ void sweep_reg(const SweepArgs& A, const LineGeom& L, T nudt)
{
    constexpr int M = 1 << LM;
    const T* in = (const T*)A.in;
    const T* dt = (const T*)L.dtab;
    const T cm = (T)L.cmul;
    T cp[M], dp[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const T nd = nudt * (dt[r] * cm);
        const T di = T(1) + T(2) * nd;
        const T lo = (r == 0) ? T(0) : ((r == M - 1) ? -T(2) * nd : -nd);
        const T up = (r == M - 1) ? T(0) : -nd;
        const T G = in[L.base + r * L.stride];
        if (r == 0) {
            const T inv = T(1) / di;
            cp[0] = up * inv;
            dp[0] = G * inv;
        } else {
            const T inv = T(1) / (di - lo * cp[r - 1]);
            cp[r] = up * inv;
            dp[r] = (G - lo * dp[r - 1]) * inv;
        }
    }
    T x = dp[M - 1];
    sweep_store<T, EPI>(A, L.base + (int64_t)(M - 1) * L.stride, x);
#pragma unroll
    for (int r = M - 2; r >= 0; --r) {
        x = dp[r] - cp[r] * x;
        sweep_store<T, EPI>(A, L.base + r * L.stride, x);
    }
}

// Long lines: Thomas with c' in the scratch vector and d' in the output (or the consumed input).
template <typename T, int EPI>
__device__ __forceinline__ void sweep_gmem(const SweepArgs& A, const LineGeom& L, T nudt, int lm)
{
    const int M = 1 << lm;
    const T* in = (const T*)A.in;
    T* dst = (EPI == EPI_STORE) ? (T*)A.out : (T*)A.in;
    T* cb = (T*)A.cbuf;
    const T* dt = (const T*)L.dtab;
    const T cm = (T)L.cmul;
    T cprev = T(0), dprev = T(0);
    for (int r = 0; r < M; ++r) {
        const int64_t idx = L.base + r * L.stride;
        const T nd = nudt * (dt[r] * cm);
        const T di = T(1) + T(2) * nd;
        const T lo = (r == 0) ? T(0) : ((r == M - 1) ? -T(2) * nd : -nd);
        const T up = (r == M - 1) ? T(0) : -nd;
        const T inv = T(1) / (di - lo * cprev);
        const T c = up * inv;
        const T dd = (in[idx] - lo * dprev) * inv;
        cb[idx] = c;
        dst[idx] = dd;
        cprev = c;
        dprev = dd;
    }
    T x = dprev;
    sweep_store<T, EPI>(A, L.base + (int64_t)(M - 1) * L.stride, x);
    for (int r = M - 2; r >= 0; --r) {
        const int64_t idx = L.base + r * L.stride;
        x = dst[idx] - cb[idx] * x;
        sweep_store<T, EPI>(A, idx, x);
    }
}

template <typename T, int EPI>
__global__ __launch_bounds__(LINE_BLOCK) void k_sweep(DevPlan P, SweepArgs A, int axis)
{
    const SweepBlk B = P.ax_blk[axis][blockIdx.x];
    const int64_t gl = B.line_start + threadIdx.x;
    if (gl >= B.line_end) return;
    const int64_t* lo = P.ax_line_off[axis];
    int k = B.k_start;
    while (gl >= lo[k + 1]) ++k;
    const UnitDev U = P.units[P.ax_units[axis][k]];
    const int64_t line = gl - lo[k];
    const LineGeom L = line_geom<T>(P, U, axis, line, B.lm);
    const T nudt = ((const T*)P.tab)[P.probs[U.prob].cst + A.nudt_sel];
    constexpr int RL = sizeof(T) == 8 ? REG_LM_F64 : REG_LM_F32;
    switch (B.lm) {
    case 0: sweep_reg<T, 0, EPI>(A, L, nudt); break;
    case 1: sweep_reg<T, 1, EPI>(A, L, nudt); break;
    case 2: sweep_reg<T, 2, EPI>(A, L, nudt); break;
    case 3: sweep_reg<T, 3, EPI>(A, L, nudt); break;
    case 4: sweep_reg<T, 4, EPI>(A, L, nudt); break;
    case 5: sweep_reg<T, 5, EPI>(A, L, nudt); break;
    case 6:
        if constexpr (RL >= 6) {
            sweep_reg<T, 6, EPI>(A, L, nudt);
            break;
        }
        [[fallthrough]];
    default: sweep_gmem<T, EPI>(A, L, nudt, B.lm); break;
    }
}

// ------------------------------------------------------------------------------------------------
// u_l(x_eval): tensor-product linear interpolation, cell min(floor(x/h), M-1); corners on a lower
// face take the payoff.  One thread per unit, FP64.
template <typename T>
__global__ void k_unit_values(DevPlan P, const T* Y, double* vals)
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
        double w = 1.0;
        bool onface = false;
        int64_t off = 0;
        int sh = 0;
        double x[MAXD];
        for (int i = 0; i < D; ++i) {
            const int upb = (corner >> i) & 1;
            w *= upb ? t[i] : 1.0 - t[i];
            const int jc = c[i] + upb;
            x[i] = (double)jc * h[i];
            if (jc == 0) onface = true;
            else off += (int64_t)(jc - 1) << sh;
            sh += U.lv[i];
        }
        const double val = onface ? payoff_at(PR, D - 1, x) : (double)Y[U.off + off];
        v += w * val;
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
// Launchers

template <typename T>
static hipError_t init_t(const DevPlan& P, void* Y, hipStream_t s)
{
    dim3 g((unsigned)P.n_node_blocks), b(NODE_BLOCK);
    switch (P.d) {
    case 2: hipLaunchKernelGGL((k_init<T, 2>), g, b, 0, s, P, (T*)Y); break;
    case 3: hipLaunchKernelGGL((k_init<T, 3>), g, b, 0, s, P, (T*)Y); break;
    case 4: hipLaunchKernelGGL((k_init<T, 4>), g, b, 0, s, P, (T*)Y); break;
    case 5: hipLaunchKernelGGL((k_init<T, 5>), g, b, 0, s, P, (T*)Y); break;
    case 6: hipLaunchKernelGGL((k_init<T, 6>), g, b, 0, s, P, (T*)Y); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init(const DevPlan& P, int prec, void* Y, hipStream_t s)
{
    if (P.total == 0) return hipSuccess;
    return prec == 0 ? init_t<double>(P, Y, s) : init_t<float>(P, Y, s);
}

template <typename T, int D>
static hipError_t stencil_td(const DevPlan& P, int op, const StencilArgs& a, hipStream_t s)
{
    dim3 g((unsigned)P.n_node_blocks), b(NODE_BLOCK);
    switch (op) {
    case OP_F_PAYOFF: hipLaunchKernelGGL((k_stencil<T, D, OP_F_PAYOFF>), g, b, 0, s, P, a); break;
    case OP_F_ZERO: hipLaunchKernelGGL((k_stencil<T, D, OP_F_ZERO>), g, b, 0, s, P, a); break;
    case OP_STAGE: hipLaunchKernelGGL((k_stencil<T, D, OP_STAGE>), g, b, 0, s, P, a); break;
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

template <typename T>
static hipError_t sweep_t(const DevPlan& P, int axis, int epi, const SweepArgs& a, hipStream_t s)
{
    dim3 g((unsigned)P.ax_nblk[axis]), b(LINE_BLOCK);
    if (epi == EPI_STORE) hipLaunchKernelGGL((k_sweep<T, EPI_STORE>), g, b, 0, s, P, a, axis);
    else hipLaunchKernelGGL((k_sweep<T, EPI_UPDATE>), g, b, 0, s, P, a, axis);
    return hipGetLastError();
}

hipError_t launch_sweep(const DevPlan& P, int prec, int axis, int epi, const SweepArgs& a,
                        hipStream_t s)
{
    if (P.ax_nblk[axis] == 0) return hipSuccess;
    return prec == 0 ? sweep_t<double>(P, axis, epi, a, s) : sweep_t<float>(P, axis, epi, a, s);
}

hipError_t launch_unit_values(const DevPlan& P, int prec, const void* Y, double* vals, hipStream_t s)
{
    if (P.n_units == 0) return hipSuccess;
    dim3 g((P.n_units + 127) / 128), b(128);
    if (prec == 0) hipLaunchKernelGGL((k_unit_values<double>), g, b, 0, s, P, (const double*)Y, vals);
    else hipLaunchKernelGGL((k_unit_values<float>), g, b, 0, s, P, (const float*)Y, vals);
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
