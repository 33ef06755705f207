// Plane-tiled ("marching") form of the time-loop operator of Sketch 1 for d <= 4, shared by the
// gfx950 kernel (amfrw_kernels.hip) and the host emulation that checks every access of a plan's
// blocks (tests/march_harness.cpp).  Everything a thread does is split into phases between block
// barriers, each written against an accessor type: buffer loads, raw pointers and LDS on the GPU,
// bounds-checked arrays on the host.
//
// A block owns one tile of the plane axes 0..d-2 of one unit (T_0 x T_1 x T_2 nodes, one node per
// thread) and walks the V axis (axis d-1) over a range of planes.  The values it needs from the
// planes j_V - 1, j_V, j_V + 1 (the tile plus a one-node halo on every plane axis) sit in a ring of
// four LDS plane slots: while the nodes of plane j_V are computed, the plane j_V + 2 (loaded into
// registers during the previous step) is written into the slot of plane j_V - 2, which no thread
// reads in that step, and plane j_V + 3 is loaded; one barrier per plane suffices and two planes are
// in flight.  Every neighbour of the 19-row stencil comes from LDS or, for the node's own column on
// the planes j_V - 1 and j_V, from registers that carry it between steps (march_cross); the unit is
// read from global memory once plus the tile halos.
//
// A halo element beyond a lower face holds 0 (the lower faces are zero in the state W = Y - g); one
// beyond an upper face holds the node below that face, the Neumann ghost u_{M+1} = u_{M-1} of
// eq. (bound1).  The stencil therefore reads every neighbour without a test; the mixed and
// advection coefficients that vanish on the upper faces are folded into the thread's coefficients.
//
// The slot strides are template constants for the full-tile shapes listed in march_shape_id (the
// LDS offsets of the stencil become instruction immediates) and run-time values for the rest.
#pragma once

#ifndef __HIPCC__
#define __host__
#define __device__
#define __forceinline__ inline
#endif

#include <algorithm>
#include <cstdint>
#include <vector>

#include "amfrw_consts.h"


namespace amf {

constexpr int MARCH_THREADS = 256;      // threads per block = nodes per tile plane (at most)
constexpr int MARCH_SEG = 32;           // V planes per block
constexpr int MARCH_SLOTS = 4;          // LDS ring of plane slots
constexpr int MARCH_DEPTH = 1;          // planes whose loads are in flight during a step (1 or 2)
constexpr int MARCH_MAX_PLANE = 1280;   // elements per plane slot (tile plus halo)
constexpr int MARCH_PF = MARCH_MAX_PLANE / MARCH_THREADS;   // prefetch registers per thread (at most)
constexpr uint32_t MARCH_NONE = 0x7FFFFFF0u;  // byte offset of a zero element: beyond every plane
constexpr int MARCH_FUSE_LM = 4;        // fused axis-1 solve: units whose axis-1 lines have <= 2^4 points

// One block of the marching operator.  lt[k] = log2 T_k for the plane axes k < d - 1 (0 beyond);
// shape = index of the compiled stride set (0: run-time strides).
struct alignas(16) MarchBlk {
    int32_t unit;
    int32_t v0;          // planes j_V = v0 + 1 .. v0 + vn (1-based)
    int32_t vn;          // 0: an empty entry (padding of the XCD-ordered table)
    int32_t o[3];        // 0-based tile origin on the plane axes
    int8_t lt[3];
    int8_t shape;
    int8_t pad_[4];
};

// log2 of the axis-0 tile width: whole lines up to 128 bytes of values (16 doubles, 32 floats), or
// 256 nodes for d = 2 (one plane axis).
inline int march_row_log2(int d, int elem) { return d == 2 ? 8 : (elem == 8 ? 4 : 5); }

// Elements of one plane slot: (T_0 + 2) x (T_1 + 2) x (T_2 + 2) over the plane axes.
inline int march_slot_elems(int d, const int* lt)
{
    int p = 1;
    for (int k = 0; k < d - 1; ++k) p *= (1 << lt[k]) + 2;
    return p;
}

// Tile extents for a unit with per-axis levels lv (d axes): nodes per tile plane <= MARCH_THREADS.
// The remaining thread budget after axis 0 is split between the other plane axes; a tile whose
// slot (with halo) would exceed MARCH_MAX_PLANE, a thin one of a unit with short axes, is halved
// along its longest axis until it fits.
inline void march_tile(int d, const int* lv, int elem, int* lt)
{
    for (int k = 0; k < 3; ++k) lt[k] = 0;
    const int na = d - 1;                                   // plane axes 0..d-2
    int budget = 8;                                         // log2 MARCH_THREADS
    lt[0] = std::min(lv[0], march_row_log2(d, elem));
    budget -= lt[0];
    if (na == 2) {
        lt[1] = std::min(lv[1], budget);
    } else if (na == 3) {
        lt[1] = std::min(lv[1], budget / 2);
        lt[2] = std::min(lv[2], budget - lt[1]);
        lt[1] = std::min(lv[1], budget - lt[2]);
    }
    while (march_slot_elems(d, lt) > MARCH_MAX_PLANE) {
        int k = 0;
        for (int i = 1; i < na; ++i)
            if (lt[i] > lt[k]) k = i;
        --lt[k];
    }
}

// Compiled stride sets: full tiles (MARCH_THREADS nodes) of d = 3 and 4 with the given log2 T_0,
// log2 T_1.  Index 0 is the run-time set.  march_dispatch maps the same indices to the types.
inline int march_shape_id(int d, const int* lt)
{
    static const int ids[][3] = {{4, 4, 2}, {4, 3, 2}, {4, 5, 1}, {4, 2, 3}, {3, 4, 4}, {3, 5, 3}};
    int sum = 0;
    for (int k = 0; k < d - 1; ++k) sum += lt[k];
    if (sum != 8) return 0;
    for (int i = 0; i < (int)(sizeof(ids) / sizeof(ids[0])); ++i)
        if (ids[i][0] == d && ids[i][1] == lt[0] && ids[i][2] == lt[1]) return i + 1;
    return 0;
}

// Blocks of a plan, unit by unit: for each V segment, its tiles in axis order, so blocks that share
// halos are adjacent.
inline void march_blocks(int d, int n_units, const int8_t* lv_of_unit /* [n_units][maxd] */, int maxd, int elem,
                         std::vector<MarchBlk>& out)
{
    for (int u = 0; u < n_units; ++u) {
        const int8_t* l8 = lv_of_unit + (size_t)u * maxd;
        int lv[8];
        for (int i = 0; i < d; ++i) lv[i] = l8[i];
        int lt[3];
        march_tile(d, lv, elem, lt);
        const int na = d - 1;
        int nt[3] = {1, 1, 1};
        for (int k = 0; k < na; ++k) nt[k] = 1 << (lv[k] - lt[k]);
        const int MV = 1 << lv[d - 1];
        const int8_t shape = (int8_t)march_shape_id(d, lt);
        for (int v0 = 0; v0 < MV; v0 += MARCH_SEG)
            for (int t2 = 0; t2 < nt[2]; ++t2)
                for (int t1 = 0; t1 < nt[1]; ++t1)
                    for (int t0 = 0; t0 < nt[0]; ++t0) {
                        MarchBlk B{};
                        B.unit = u;
                        B.v0 = v0;
                        B.vn = std::min(MARCH_SEG, MV - v0);
                        B.o[0] = t0 << lt[0];
                        B.o[1] = t1 << lt[1];
                        B.o[2] = t2 << lt[2];
                        for (int k = 0; k < 3; ++k) B.lt[k] = (int8_t)lt[k];
                        B.shape = shape;
                        out.push_back(B);
                    }
    }
}

// The blocks of march_blocks reordered for a device that deals blocks to its nx XCDs round-robin
// (block b to XCD b mod nx).  The blocks of one (unit, V range), which share their halo planes, stay
// together and in order on one XCD, so that they run close in time and each halo plane is read from
// HBM once into that XCD's L2.  The groups go, longest first, to the XCD with the least work so far
// (work = the planes a block reads), and each XCD's queue is padded with empty blocks (vn = 0) to
// the longest queue.
inline void march_order_xcd(const std::vector<MarchBlk>& in, int nx, std::vector<MarchBlk>& out)
{
    struct Group {
        size_t first, n;
        int64_t work;
    };
    std::vector<Group> groups;
    for (size_t i = 0; i < in.size();) {
        size_t j = i;
        int64_t w = 0;
        for (; j < in.size() && in[j].unit == in[i].unit && in[j].v0 == in[i].v0; ++j) w += in[j].vn + 2;
        groups.push_back({i, j - i, w});
        i = j;
    }
    std::stable_sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) { return a.work > b.work; });
    std::vector<std::vector<MarchBlk>> q((size_t)nx);
    std::vector<int64_t> load((size_t)nx, 0);
    for (const Group& g : groups) {
        const size_t x = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
        for (size_t k = 0; k < g.n; ++k) q[x].push_back(in[g.first + k]);
        load[x] += g.work;
    }
    size_t len = 0;
    for (const auto& v : q) len = std::max(len, v.size());
    out.assign(len * (size_t)nx, MarchBlk{});
    for (size_t x = 0; x < (size_t)nx; ++x)
        for (size_t k = 0; k < q[x].size(); ++k) out[k * (size_t)nx + x] = q[x][k];
}

// Geometry of one block, shared by all its threads.
template <int D>
struct MarchGeo {
    int M[D];            // extents of the unit's axes
    int64_t E[D];        // strides (1 << sum of lower levels)
    int64_t off;         // unit offset in every grid vector
    int o[3], T[3], H[3];  // tile origin, extent and stored extent (with halo; 1 for absent axes)
    int S1, S2, LP;      // element strides of axes 1, 2 inside a slot; elements of a slot
    int v0, vn;
    int nact;            // active threads (tile nodes)
};

template <int D>
__host__ __device__ __forceinline__ void march_geo(const int8_t* lv, int64_t off, const MarchBlk& B, MarchGeo<D>& G)
{
    int64_t e = 1;
    for (int i = 0; i < D; ++i) {
        G.M[i] = 1 << lv[i];
        G.E[i] = e;
        e <<= lv[i];
    }
    G.off = off;
    G.nact = 1;
    for (int k = 0; k < 3; ++k) {
        G.o[k] = B.o[k];
        G.T[k] = 1 << B.lt[k];
        G.H[k] = k >= D - 1 ? 1 : G.T[k] + 2;
        if (k < D - 1) G.nact *= G.T[k];
    }
    G.S1 = G.H[0];
    G.S2 = G.H[0] * G.H[1];
    G.LP = G.S2 * G.H[2];
    G.v0 = B.v0;
    G.vn = B.vn;
}

// Stride sets.  MarchRt reads the block's geometry; MarchCt<D, L0, L1> is the full tile with
// T_0 = 2^L0, T_1 = 2^L1 (d >= 3) and T_2 = MARCH_THREADS / (T_0 T_1) (d = 4).
struct MarchRt {
    static constexpr int NPF = MARCH_PF;
    static constexpr bool FULL = false;
    template <int D>
    __host__ __device__ static int t0(const MarchGeo<D>& G) { return G.T[0]; }
    template <int D>
    __host__ __device__ static int t1(const MarchGeo<D>& G) { return G.T[1]; }
    template <int D>
    __host__ __device__ static int s1(const MarchGeo<D>& G) { return G.S1; }
    template <int D>
    __host__ __device__ static int s2(const MarchGeo<D>& G) { return G.S2; }
    template <int D>
    __host__ __device__ static int lp(const MarchGeo<D>& G) { return G.LP; }
};

template <int DD, int L0, int L1>
struct MarchCt {
    static constexpr int T0 = 1 << L0, T1 = DD >= 3 ? 1 << L1 : 1, T2 = DD == 4 ? MARCH_THREADS / (T0 * T1) : 1;
    static constexpr int H0 = T0 + 2, H1 = DD >= 3 ? T1 + 2 : 1, H2 = DD == 4 ? T2 + 2 : 1;
    static constexpr int LPC = H0 * H1 * H2;
    static constexpr int NPF = (LPC + MARCH_THREADS - 1) / MARCH_THREADS;
    static constexpr bool FULL = true;
    static_assert(T0 * T1 * T2 == MARCH_THREADS && LPC <= MARCH_MAX_PLANE, "full tiles that fit a slot");
    template <int D>
    __host__ __device__ static constexpr int t0(const MarchGeo<D>&) { return T0; }
    template <int D>
    __host__ __device__ static constexpr int t1(const MarchGeo<D>&) { return T1; }
    template <int D>
    __host__ __device__ static constexpr int s1(const MarchGeo<D>&) { return H0; }
    template <int D>
    __host__ __device__ static constexpr int s2(const MarchGeo<D>&) { return H0 * H1; }
    template <int D>
    __host__ __device__ static constexpr int lp(const MarchGeo<D>&) { return LPC; }
};

// Calls f with the stride set of a block's shape index (the indices of march_shape_id).
template <int D, class F>
__host__ __device__ __forceinline__ void march_dispatch(int shape, F&& f)
{
    if constexpr (D == 4) {
        switch (shape) {
        case 1: f(MarchCt<4, 4, 2>{}); return;
        case 2: f(MarchCt<4, 3, 2>{}); return;
        case 3: f(MarchCt<4, 5, 1>{}); return;
        case 4: f(MarchCt<4, 2, 3>{}); return;
        default: break;
        }
    } else if constexpr (D == 3) {
        switch (shape) {
        case 5: f(MarchCt<3, 4, 4>{}); return;
        case 6: f(MarchCt<3, 5, 3>{}); return;
        default: break;
        }
    }
    f(MarchRt{});
}

// Per-thread state kept across phases: its node in the tile, the coefficient products of its node
// on the plane axes (fixed while the thread walks V), the byte offsets (inside one V plane) of the
// slot elements it fetches.
template <typename T, int D, int NPF>
struct MarchThr {
    int x[3];            // position in the tile
    int j[3];            // 1-based node index on the plane axes
    bool active;
    bool top[3];         // on the upper face of a plane axis
    int c;               // its element inside a slot
    uint32_t gob;        // byte offset of its node inside a V plane of the unit
    T fmask;             // 0 on a Dirichlet rate face (eq bound1_0), else 1
    T tdiff[3], adv[3];
    T cpair[3];          // rho_ik tmix_i tmix_k for the plane-axis pairs (0,1), (0,2), (1,2); 0 on a face
    T cv[3];             // sigma phi_i tmix_i tmix_V for the pairs (i, V); 0 on a face
    uint32_t pfb[NPF];   // byte offsets in a V plane of the fetched slot elements (MARCH_NONE: zero)
};

__host__ __device__ __forceinline__ int march_pair(int i, int k) { return i + k - 1; }   // (0,1)->0 (0,2)->1 (1,2)->2

template <typename T, int D, class Sh, int NPF>
__host__ __device__ __forceinline__ void march_thread(const MarchGeo<D>& G, int tid, MarchThr<T, D, NPF>& t)
{
    const int T0 = Sh::t0(G), T1 = Sh::t1(G);
    const int S[3] = {1, Sh::s1(G), Sh::s2(G)};
    const int LP = Sh::lp(G);
    t.active = Sh::FULL || tid < G.nact;
    const int tt = t.active ? tid : 0;
    t.x[0] = tt & (T0 - 1);
    t.x[1] = (tt / T0) & (T1 - 1);
    t.x[2] = tt / (T0 * T1);
    for (int k = 0; k < 3; ++k) {
        t.j[k] = G.o[k] + t.x[k] + 1;
        t.top[k] = k < D - 1 && t.j[k] == G.M[k];
    }
    t.c = 0;
    int64_t rel = 0;
    for (int k = 0; k < D - 1; ++k) {
        t.c += (t.x[k] + 1) * S[k];
        rel += (int64_t)(t.j[k] - 1) * G.E[k];
    }
    t.gob = (uint32_t)(rel * (int64_t)sizeof(T));
    // slot elements this thread fetches: e = tid + r * MARCH_THREADS at stored position y (y = 0 is
    // the halo before the tile), node jj = o + y: 0 is the lower face (zero), M + 1 the ghost of the
    // upper face (node M - 1; the lower face when M = 1)
    for (int r = 0; r < NPF; ++r) {
        const int e = tid + r * MARCH_THREADS;
        t.pfb[r] = MARCH_NONE;
        if (e >= LP) continue;
        const int y[3] = {e % S[1], D >= 3 ? (e / S[1]) % (S[2] / S[1]) : 0, D == 4 ? e / S[2] : 0};
        bool zero = false;
        int64_t off = 0;
        for (int k = 0; k < D - 1; ++k) {
            int jj = G.o[k] + y[k];
            if (jj == G.M[k] + 1) jj = G.M[k] - 1;
            zero = zero || jj < 1;
            off += (int64_t)(jj - 1) * G.E[k];
        }
        if (!zero) t.pfb[r] = (uint32_t)(off * (int64_t)sizeof(T));
    }
}

// Coefficient factors of the plane axes and the pairs (tables as in the streaming operator).
template <typename T, int D, int NPF, class Mem>
__host__ __device__ __forceinline__ void march_coefs(const MarchGeo<D>& G, const int32_t* utab, const T* tab,
                                                     const T* cst, MarchThr<T, D, NPF>& t, Mem& m)
{
    T tmix[3], tphi[3];
    for (int k = 0; k < 3; ++k) {
        t.tdiff[k] = T(0);
        t.adv[k] = T(0);
        t.cpair[k] = T(0);
        t.cv[k] = T(0);
        tmix[k] = T(0);
        tphi[k] = T(0);
    }
    for (int k = 0; k < D - 1; ++k) {
        const T* tk = tab + utab[k];
        const int Mk = G.M[k], jk = t.j[k];
        t.tdiff[k] = m.tab(tk, jk - 1);
        tmix[k] = m.tab(tk, Mk + jk - 1);
        tphi[k] = m.tab(tk, 2 * Mk + jk - 1);
    }
    // advection of paper axes 2..N-1 (plane axes 1..d-2), zero on the upper face
    for (int k = 1; k < D - 1; ++k) {
        if (t.j[k] == G.M[k]) continue;
        T s = T(0);
        for (int jj = 1; jj <= k; ++jj) s += m.tab(cst, CST_RHO + k * MAXD + jj) * tphi[jj];
        t.adv[k] = tmix[k] * s;
    }
    const T* tV = tab + utab[D - 1];
    const T tmixV = m.tab(tV, G.M[D - 1] + 1);
    for (int i = 0; i < D - 1; ++i) {
        for (int k = i + 1; k < D - 1; ++k)
            t.cpair[march_pair(i, k)] =
                (t.top[i] || t.top[k]) ? T(0) : m.tab(cst, CST_RHO + i * MAXD + k) * tmix[i] * tmix[k];
        t.cv[i] = t.top[i] ? T(0) : m.tab(cst, CST_SPHI + i) * tmix[i] * tmixV;
    }
}

// Dirichlet rate faces (eq bound1_0): rows of boundary data.
template <typename T, int D, int NPF>
__host__ __device__ __forceinline__ void march_face(int dirichlet, MarchThr<T, D, NPF>& t)
{
    bool face = false;
    for (int k = 0; k < D - 1; ++k) face = face || (dirichlet && t.top[k]);
    t.fmask = face ? T(0) : T(1);
}

// Fused axis-1 solve (units with M_1 <= 2^MARCH_FUSE_LM, so a tile row is a whole axis-1 line):
// element offset of this thread's row in the unit's axis-1 Thomas factor block for V plane jv
// (1-based).  The block holds, per V plane, inv (M_1), a inv (M_1) and c' (M_1).
template <typename T, int D, int NPF>
__host__ __device__ __forceinline__ int march_fac_at(const MarchGeo<D>& G, int jv, const MarchThr<T, D, NPF>& t)
{
    return (jv - 1) * 3 * G.M[0] + (t.j[0] - 1);
}

template <int D>
__host__ __device__ __forceinline__ bool march_fused(const MarchGeo<D>& G, bool fuse)
{
    return fuse && G.M[0] <= (1 << MARCH_FUSE_LM);
}

// Element range of V plane jv (1-based) of a unit inside a grid vector: its first element and its
// length; planes outside 1..M_V (plane 0 is the lower face) have length 0, so every fetch from them
// yields 0.
template <int D>
__host__ __device__ __forceinline__ int64_t march_plane_base(const MarchGeo<D>& G, int jv)
{
    return G.off + (jv >= 1 && jv <= G.M[D - 1] ? (int64_t)(jv - 1) * G.E[D - 1] : 0);
}

template <int D>
__host__ __device__ __forceinline__ int64_t march_plane_len(const MarchGeo<D>& G, int jv)
{
    return jv >= 1 && jv <= G.M[D - 1] ? G.E[D - 1] : 0;
}

// Prefetch registers of one plane: this thread's share of the slot, as loaded (x0 from X0 and, for
// OP_STAGE2, x1 from X1; the stage combination X0 + a X1 is formed when the values go to LDS, so no
// instruction between the load and the stash waits for the load).
template <typename T, int OP, int NPF>
struct MarchPf {
    T x0[NPF];
    T x1[OP == OP_STAGE2 ? NPF : 1];
};

// Global -> registers: this thread's share of the slot of plane jv.  With live = false the loads are
// still issued but read nothing (a zero-length range): the loop then issues the same loads on every
// step, which keeps the wait counts exact.
template <typename T, int D, int OP, int NPF, class Mem>
__host__ __device__ __forceinline__ void march_fetch(const MarchGeo<D>& G, int jv, const T* X0, const T* X1,
                                                     const MarchThr<T, D, NPF>& t, MarchPf<T, OP, NPF>& pf, Mem& m,
                                                     bool live = true)
{
    const int64_t b = march_plane_base<D>(G, jv), n = live ? march_plane_len<D>(G, jv) : 0;
    const auto h0 = m.plane(X0, b, n);
#pragma unroll
    for (int r = 0; r < NPF; ++r) pf.x0[r] = m.pld(h0, t.pfb[r]);
    if constexpr (OP == OP_STAGE2) {
        const auto h1 = m.plane(X1, b, n);
#pragma unroll
        for (int r = 0; r < NPF; ++r) pf.x1[r] = m.pld(h1, t.pfb[r]);
    }
}

// The V^2 factors of the block's planes (table entries v0 .. v0 + vn - 1), loaded once into the LDS
// words after the slot ring, so that the plane loop reads them from LDS: a global load there would
// make the step wait for the plane prefetch issued before it.
template <typename T, int D, class Sh, class Mem>
__host__ __device__ __forceinline__ void march_vsq(const MarchGeo<D>& G, int tid, const T* tV, Mem& m)
{
    if (tid < G.vn) m.sw(MARCH_SLOTS * Sh::lp(G) + tid, m.tab(tV, G.v0 + tid));
}

template <typename T, int D, class Sh, class Mem>
__host__ __device__ __forceinline__ T march_vsq_of(const MarchGeo<D>& G, int s, Mem& m)
{
    return m.sr(MARCH_SLOTS * Sh::lp(G) + s - 1);
}

// Registers -> the LDS slot of plane jv (OP_STAGE2: X0 + a X1).
template <typename T, int D, class Sh, int OP, int NPF, class Mem>
__host__ __device__ __forceinline__ void march_stash(const MarchGeo<D>& G, int tid, int jv,
                                                     const MarchPf<T, OP, NPF>& pf, T a, Mem& m)
{
    const int LP = Sh::lp(G);
    const int base = (jv & (MARCH_SLOTS - 1)) * LP;
#pragma unroll
    for (int r = 0; r < NPF; ++r) {
        const int e = tid + r * MARCH_THREADS;
        if (e < LP) {
            if constexpr (OP == OP_STAGE2) m.sw(base + e, pf.x0[r] + a * pf.x1[r]);
            else m.sw(base + e, pf.x0[r]);
        }
    }
}

// The "cross" of this thread's node on plane jv: the node and its two neighbours along each plane
// axis, x[0] = centre, x[1 + 2i] = node - e_i, x[2 + 2i] = node + e_i.  A thread keeps the crosses
// of planes jv - 1 and jv in registers while it walks V, so each step reads only the cross of plane
// jv + 1 and the in-plane diagonal neighbours of plane jv from LDS (19 values for d = 4, not 33).
template <int D>
struct MarchX {
    static constexpr int N = 2 * D - 1;
};

template <typename T, int D, class Sh, int NPF, class Mem>
__host__ __device__ __forceinline__ void march_cross(const MarchGeo<D>& G, const MarchThr<T, D, NPF>& t, int jv,
                                                     T (&x)[MarchX<D>::N], Mem& m)
{
    const int S[3] = {1, Sh::s1(G), Sh::s2(G)};
    const int sc = (jv & (MARCH_SLOTS - 1)) * Sh::lp(G) + t.c;
    x[0] = m.sr(sc);
#pragma unroll
    for (int i = 0; i < D - 1; ++i) {
        x[1 + 2 * i] = m.sr(sc - S[i]);
        x[2 + 2 * i] = m.sr(sc + S[i]);
    }
}

// Sketch 1 with zero lower faces at this thread's node of plane jv, from the crosses of planes
// jv - 1, jv, jv + 1 (xm, xc, xp; xp is not read on the V face) and the diagonal neighbours of the
// LDS slot of plane jv: second differences (the upper-face ghosts are stored in the halo), mixed
// differences for every pair (zero on either upper face: folded into cpair and cv), advection on the
// plane axes 1..d-2 (zero on the upper face: folded into adv).  Returns F before the stage
// combination (vsq = V^2 of the plane, tdV = sigma^2 / (2 h_V^2)); 0 on a Dirichlet rate face.
// The only branch is on the V face, uniform over the block.
template <typename T, int D, class Sh, int NPF, class Mem>
__host__ __device__ __forceinline__ T march_F(const MarchGeo<D>& G, const MarchThr<T, D, NPF>& t, int jv, T vsq,
                                              T tdV, const T (&xm)[MarchX<D>::N], const T (&xc)[MarchX<D>::N],
                                              const T (&xp)[MarchX<D>::N], Mem& m)
{
    const int S[3] = {1, Sh::s1(G), Sh::s2(G)};
    const int sc = (jv & (MARCH_SLOTS - 1)) * Sh::lp(G) + t.c;
    const T c0 = xc[0];
    const bool vtop = jv == G.M[D - 1];                      // uniform over the block
    const T vm = xm[0];
    const T vp = vtop ? vm : xp[0];
    T acc = tdV * (vp - T(2) * c0 + vm);
#pragma unroll
    for (int i = 0; i < D - 1; ++i) {
        const T lo = xc[1 + 2 * i];
        const T hi = xc[2 + 2 * i];
        acc += t.tdiff[i] * (hi - T(2) * c0 + lo);
        if (i > 0) acc += t.adv[i] * (hi - lo);             // no advection term on axis 0
#pragma unroll
        for (int k = i + 1; k < D - 1; ++k) {
            const T xx = m.sr(sc + S[i] + S[k]) + m.sr(sc - S[i] - S[k]) - m.sr(sc + S[i] - S[k]) -
                         m.sr(sc - S[i] + S[k]);
            acc += t.cpair[march_pair(i, k)] * xx;
        }
    }
    if (!vtop) {
#pragma unroll
        for (int i = 0; i < D - 1; ++i) {
            const T xx = xp[2 + 2 * i] + xm[1 + 2 * i] - xm[2 + 2 * i] - xp[1 + 2 * i];
            acc += t.cv[i] * xx;
        }
    }
    return t.fmask * vsq * acc;
}

}  // namespace amf
