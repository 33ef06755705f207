// Plane-tiled ("marching") form of the time-loop operator of Sketch 1 for d <= 4, shared by the
// gfx950 kernel (amfrw_kernels.hip) and the host emulation that checks every access of a plan's
// blocks (tests/march_harness.cpp).  Everything a thread does is split into phases between block
// barriers, each written against an accessor type: raw pointers and LDS on the GPU, bounds-checked
// arrays on the host.
//
// A block owns one tile of the plane axes 0..d-2 of one unit (T_0 x T_1 x T_2 nodes, one node per
// thread) and walks the V axis (axis d-1) over a range of planes.  The values it needs from the
// planes j_V - 1, j_V, j_V + 1 (the tile plus a one-node halo on every plane axis) sit in a ring of
// four LDS plane slots: while the nodes of plane j_V are computed from three slots, the plane
// j_V + 2 is loaded into registers and then written into the fourth slot, which no thread reads in
// that step, so one barrier per plane suffices.  Every neighbour read of the 19-row stencil then
// comes from LDS; the unit is read from global memory once plus the tile halos.
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
constexpr int MARCH_MAX_PLANE = 1280;   // elements per plane slot, tile plus halo plus 2 pads
constexpr int MARCH_PF = MARCH_MAX_PLANE / MARCH_THREADS;   // prefetch registers per thread

// One block of the marching operator.  lt[k] = log2 T_k for the plane axes k < d - 1 (0 beyond);
// h0 = 1 when the tile holds part of its axis-0 lines (a one-node halo on axis 0), 0 when it holds
// whole lines (no axis-0 halo: the line ends are faces).
struct alignas(16) MarchBlk {
    int32_t unit;
    int32_t v0;          // planes j_V = v0 + 1 .. v0 + vn (1-based)
    int32_t vn;
    int32_t o[3];        // 0-based tile origin on the plane axes
    int8_t lt[3];
    int8_t h0;
    int8_t pad_[4];
};

// Tile extents for a unit with per-axis levels lv (d axes): nodes per tile plane <= MARCH_THREADS.
// Axis 0 takes whole lines up to RW = 256 bytes of values (32 doubles, 64 floats; 256 nodes for
// d = 2), else RW-node pieces: either way the 32 (FP64) or 64 (FP32) lanes that the LDS serves
// together read 256 consecutive bytes, which spread over all 64 banks.  The rest of the threads go to
// axes 1..d-2, as evenly as their extents allow.
inline void march_tile(int d, const int* lv, int elem, int* lt, int* h0)
{
    for (int k = 0; k < 3; ++k) lt[k] = 0;
    const int na = d - 1;                                   // plane axes 0..d-2
    int budget = 8;                                         // log2 MARCH_THREADS
    const int rw = na == 1 ? 8 : (elem == 8 ? 5 : 6);       // log2 of the row width in nodes
    lt[0] = std::min(lv[0], rw);
    *h0 = lt[0] < lv[0] ? 1 : 0;
    budget -= lt[0];
    if (na == 2) {
        lt[1] = std::min(lv[1], budget);
    } else if (na == 3) {
        lt[1] = std::min(lv[1], budget / 2);
        lt[2] = std::min(lv[2], budget - lt[1]);
        lt[1] = std::min(lv[1], budget - lt[2]);
    }
}

// Elements of one plane slot: (T_0 + 2 h0) x (T_1 + 2) x (T_2 + 2) over the plane axes, plus a
// leading and a trailing pad element (so that axis-0 neighbours of whole-line tiles stay inside).
inline int march_slot_elems(int d, const int* lt, int h0)
{
    int p = (1 << lt[0]) + 2 * h0;
    for (int k = 1; k < d - 1; ++k) p *= (1 << lt[k]) + 2;
    return p + 2;
}

// Blocks of a plan, unit by unit: for each V segment, its tiles in axis order, so blocks that share
// halos are adjacent (and land on the same XCD).
inline void march_blocks(int d, int n_units, const int8_t* lv_of_unit /* [n_units][maxd] */, int maxd, int elem,
                         std::vector<MarchBlk>& out)
{
    for (int u = 0; u < n_units; ++u) {
        const int8_t* l8 = lv_of_unit + (size_t)u * maxd;
        int lv[8];
        for (int i = 0; i < d; ++i) lv[i] = l8[i];
        int lt[3], h0;
        march_tile(d, lv, elem, lt, &h0);
        const int na = d - 1;
        int nt[3] = {1, 1, 1};
        for (int k = 0; k < na; ++k) nt[k] = 1 << (lv[k] - lt[k]);
        const int MV = 1 << lv[d - 1];
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
                        B.h0 = (int8_t)h0;
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
    int h0;              // axis-0 halo width (0 or 1)
    int S1, S2, LP;      // element strides of axes 1, 2; tile elements of a slot (without pads)
    int SLOT;            // slot size: LP + 2 pads
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
    G.h0 = B.h0;
    for (int k = 0; k < 3; ++k) {
        G.o[k] = B.o[k];
        G.T[k] = 1 << B.lt[k];
        G.H[k] = k >= D - 1 ? 1 : (k == 0 ? G.T[0] + 2 * G.h0 : G.T[k] + 2);
        if (k < D - 1) G.nact *= G.T[k];
    }
    G.S1 = G.H[0];
    G.S2 = G.H[0] * G.H[1];
    G.LP = G.S2 * G.H[2];
    G.SLOT = G.LP + 2;
    G.v0 = B.v0;
    G.vn = B.vn;
}

// Per-thread state kept across phases: its node in the tile, the coefficient products of its node
// on the plane axes (fixed while the thread walks V), the offsets (inside one V plane) of the slot
// elements it fetches, and the prefetch registers.
template <typename T, int D>
struct MarchThr {
    int x[3];            // position in the tile
    int j[3];            // 1-based node index on the plane axes
    bool active;
    bool top[3];         // on the upper face of a plane axis
    int c;               // its element inside a slot (pads included)
    int64_t g0;          // its global index in plane j_V = 1
    T m0;                // 0 when its axis-0 lower neighbour is the lower face of a whole-line tile
    T fmask;             // 0 on a Dirichlet rate face (eq bound1_0), else 1
    T tdiff[3], adv[3];
    T cpair[3];          // rho_ik tmix_i tmix_k for the plane-axis pairs (0,1), (0,2), (1,2); 0 on a face
    T cv[3];             // sigma phi_i tmix_i tmix_V for the pairs (i, V); 0 on a face
    int32_t pfo[MARCH_PF];  // offsets in a V plane of the fetched slot elements (-1: zero)
    T pf[MARCH_PF];
};

__host__ __device__ __forceinline__ int march_pair(int i, int k) { return i + k - 1; }   // (0,1)->0 (0,2)->1 (1,2)->2

template <typename T, int D>
__host__ __device__ __forceinline__ void march_thread(const MarchGeo<D>& G, int tid, MarchThr<T, D>& t)
{
    t.active = tid < G.nact;
    const int tt = t.active ? tid : 0;
    t.x[0] = tt & (G.T[0] - 1);
    t.x[1] = (tt / G.T[0]) & (G.T[1] - 1);
    t.x[2] = tt / (G.T[0] * G.T[1]);
    for (int k = 0; k < 3; ++k) {
        t.j[k] = G.o[k] + t.x[k] + 1;
        t.top[k] = k < D - 1 && t.j[k] == G.M[k];
    }
    const int S[3] = {1, G.S1, G.S2};
    t.c = 1 + t.x[0] + G.h0;
    t.g0 = G.off;
    for (int k = 0; k < D - 1; ++k) {
        if (k > 0) t.c += (t.x[k] + 1) * S[k];
        t.g0 += (int64_t)(t.j[k] - 1) * G.E[k];
    }
    t.m0 = (G.h0 == 0 && t.x[0] == 0) ? T(0) : T(1);
    // slot elements this thread fetches: e = tid + r * MARCH_THREADS at stored position y, node
    // jj = o + y (axes with a halo: y = 0 is the halo before the tile) or y + 1 (whole axis-0
    // lines); 0 outside the unit
    for (int r = 0; r < MARCH_PF; ++r) {
        const int e = tid + r * MARCH_THREADS;
        t.pfo[r] = -1;
        if (e >= G.LP) continue;
        const int y[3] = {e % G.H[0], (e / G.H[0]) % G.H[1], e / G.S2};
        bool ok = true;
        int64_t rel = 0;
        for (int k = 0; k < D - 1; ++k) {
            const int jj = G.o[k] + y[k] + (k == 0 ? 1 - G.h0 : 0);
            ok = ok && jj >= 1 && jj <= G.M[k];
            rel += (int64_t)(jj - 1) * G.E[k];
        }
        if (ok) t.pfo[r] = (int32_t)rel;
    }
}

// Coefficient factors of the plane axes and the pairs (tables as in the streaming operator).
template <typename T, int D, class Mem>
__host__ __device__ __forceinline__ void march_coefs(const MarchGeo<D>& G, const int32_t* utab, const T* tab,
                                                     const T* cst, MarchThr<T, D>& t, Mem& m)
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
template <typename T, int D>
__host__ __device__ __forceinline__ void march_face(int dirichlet, MarchThr<T, D>& t)
{
    bool face = false;
    for (int k = 0; k < D - 1; ++k) face = face || (dirichlet && t.top[k]);
    t.fmask = face ? T(0) : T(1);
}

// Global -> registers: this thread's share of the slot of plane jv (0 for elements beyond the unit's
// faces; plane 0 is the lower face).  OP_STAGE2 stages X0 + a X1.  Only lanes whose element lies in
// the slot and inside the unit load: the rest keep 0 without touching memory.
template <typename T, int D, int OP, class Mem>
__host__ __device__ __forceinline__ void march_fetch(const MarchGeo<D>& G, int jv, const T* X0, const T* X1, T a,
                                                     MarchThr<T, D>& t, Mem& m)
{
    const bool vok = jv >= 1 && jv <= G.M[D - 1];
    const int64_t vb = G.off + (int64_t)(jv - 1) * G.E[D - 1];
#pragma unroll
    for (int r = 0; r < MARCH_PF; ++r) {
        T v = T(0);
        if (vok && t.pfo[r] >= 0) {
            v = m.ld(X0, vb + t.pfo[r]);
            if constexpr (OP == OP_STAGE2) v += a * m.ld(X1, vb + t.pfo[r]);
        }
        t.pf[r] = v;
    }
}

// Registers -> the LDS slot of plane jv.
template <typename T, int D, class Mem>
__host__ __device__ __forceinline__ void march_stash(const MarchGeo<D>& G, int tid, int jv, const MarchThr<T, D>& t,
                                                     Mem& m)
{
    const int base = (jv & (MARCH_SLOTS - 1)) * G.SLOT + 1;
#pragma unroll
    for (int r = 0; r < MARCH_PF; ++r) {
        const int e = tid + r * MARCH_THREADS;
        if (e < G.LP) m.sw(base + e, t.pf[r]);
    }
}

// The pads of every slot hold 0 (written once, before the first barrier, by the first threads).
template <typename T, int D, class Mem>
__host__ __device__ __forceinline__ void march_pads(const MarchGeo<D>& G, int tid, Mem& m)
{
    if (tid < 2 * MARCH_SLOTS) m.sw((tid >> 1) * G.SLOT + (tid & 1) * (G.SLOT - 1), T(0));
}

// Sketch 1 with zero lower faces at this thread's node of plane jv, from the LDS slots of planes
// jv - 1, jv, jv + 1: second differences (Neumann ghost on the upper faces), mixed differences for
// every pair (zero on either upper face: folded into cpair and cv), advection on the plane axes
// 1..d-2 (zero on the upper face: folded into adv).  Returns F before the stage combination
// (vsq = V^2 of the plane, tdV = sigma^2 / (2 h_V^2)); 0 on a Dirichlet rate face.  c0 receives the
// node's own value.  No branch depends on the lane: reads beyond a face land on stored zeros, halo
// or pad elements and are then ignored or multiplied by 0.
template <typename T, int D, class Mem>
__host__ __device__ __forceinline__ T march_F(const MarchGeo<D>& G, const MarchThr<T, D>& t, int jv, T vsq, T tdV,
                                              T& c0, Mem& m)
{
    const int sm = ((jv - 1) & (MARCH_SLOTS - 1)) * G.SLOT + t.c, sc = (jv & (MARCH_SLOTS - 1)) * G.SLOT + t.c,
              sp = ((jv + 1) & (MARCH_SLOTS - 1)) * G.SLOT + t.c;
    const int S[3] = {1, G.S1, G.S2};
    const T m0 = t.m0;
    c0 = m.sr(sc);
    const bool vtop = jv == G.M[D - 1];                      // uniform over the block
    const T vm = m.sr(sm);
    const T vp = vtop ? vm : m.sr(sp);
    T acc = tdV * (vp - T(2) * c0 + vm);
#pragma unroll
    for (int i = 0; i < D - 1; ++i) {
        const T li = i == 0 ? m0 : T(1);
        const T xm = li * m.sr(sc - S[i]);
        const T xr = m.sr(sc + S[i]);
        const T xp = t.top[i] ? xm : xr;
        acc += t.tdiff[i] * (xp - T(2) * c0 + xm) + t.adv[i] * (xp - xm);
#pragma unroll
        for (int k = i + 1; k < D - 1; ++k) {
            const T xx = m.sr(sc + S[i] + S[k]) + li * m.sr(sc - S[i] - S[k]) - m.sr(sc + S[i] - S[k]) -
                         li * m.sr(sc - S[i] + S[k]);
            acc += t.cpair[march_pair(i, k)] * xx;
        }
    }
    if (!vtop) {
#pragma unroll
        for (int i = 0; i < D - 1; ++i) {
            const T li = i == 0 ? m0 : T(1);
            const T xx = m.sr(sp + S[i]) + li * m.sr(sm - S[i]) - m.sr(sm + S[i]) - li * m.sr(sp - S[i]);
            acc += t.cv[i] * xx;
        }
    }
    return t.fmask * vsq * acc;
}

// Global index of this thread's node in plane jv.
template <int D, typename TT>
__host__ __device__ __forceinline__ int64_t march_index(const MarchGeo<D>& G, const TT& t, int jv)
{
    return t.g0 + (int64_t)(jv - 1) * G.E[D - 1];
}

}  // namespace amf
