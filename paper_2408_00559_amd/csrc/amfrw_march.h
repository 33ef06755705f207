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
constexpr int MARCH_MAX_PLANE = 1024;   // elements per plane slot, tile plus halo
constexpr int MARCH_PF = MARCH_MAX_PLANE / MARCH_THREADS;   // prefetch registers per thread

// One block of the marching operator.  lt[k] = log2 T_k for the plane axes k < d - 1 (0 beyond).
struct alignas(16) MarchBlk {
    int32_t unit;
    int32_t v0;          // planes j_V = v0 + 1 .. v0 + vn (1-based)
    int32_t vn;
    int32_t o[3];        // 0-based tile origin on the plane axes
    int8_t lt[3];
    int8_t pad_[5];
};

// Tile extents for a unit with per-axis levels lv (d axes): nodes per tile plane <= MARCH_THREADS,
// axis 0 up to 128 bytes of values, the rest spread over axes 1..d-2; the halo plane must fit a slot.
inline void march_tile(int d, const int* lv, int elem, int* lt)
{
    for (int k = 0; k < 3; ++k) lt[k] = 0;
    const int na = d - 1;                                   // plane axes 0..d-2
    int budget = 8;                                         // log2 MARCH_THREADS
    const int t0max = elem == 8 ? 4 : 5;                    // 16 doubles / 32 floats
    lt[0] = std::min({lv[0], na == 1 ? budget : t0max, budget});
    budget -= lt[0];
    if (na >= 2) {
        if (na == 2) {
            lt[1] = std::min(lv[1], budget);
        } else {
            lt[1] = std::min(lv[1], budget / 2);
            lt[2] = std::min(lv[2], budget - lt[1]);
            lt[1] = std::min(lv[1], budget - lt[2]);
        }
    }
    // the halo plane must fit a slot (only long axis-0 tiles of d = 2 can reach it)
    auto plane = [&] {
        int p = 1;
        for (int k = 0; k < na && k < 3; ++k) p *= (1 << lt[k]) + 2;
        return p;
    };
    while (plane() > MARCH_MAX_PLANE && lt[0] > 0) --lt[0];
}

// Blocks of a plan, unit by unit (units given as levels and counts): for each V segment, its tiles
// in axis order, so blocks that share halos are adjacent (and land on the same XCD).
inline void march_blocks(int d, int n_units, const int8_t* lv_of_unit /* [n_units][MAXD] */, int maxd, int elem,
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
                        out.push_back(B);
                    }
    }
}

// Geometry of one block, shared by all its threads.
template <int D>
struct MarchGeo {
    int M[D];            // extents of the unit's axes
    int64_t E[D];        // strides (1 << sum of lower levels)
    int64_t off;         // unit offset in every grid vector
    int o[3], T[3], H[3];  // tile origin, extent and halo extent (T + 2, or 1 for absent axes)
    int S1, S2, LP;      // slot strides and slot size
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
        G.H[k] = k < D - 1 ? G.T[k] + 2 : 1;
        if (k < D - 1) G.nact *= G.T[k];
    }
    G.S1 = G.H[0];
    G.S2 = G.H[0] * G.H[1];
    G.LP = G.S2 * G.H[2];
    G.v0 = B.v0;
    G.vn = B.vn;
}

// Per-thread state kept across phases: its node in the tile, the 1-D coefficient factors of the
// plane axes (fixed while the thread walks V) and the prefetch registers.
template <typename T, int D>
struct MarchThr {
    int x[3];            // position in the tile
    int j[3];            // 1-based node index on the plane axes
    bool active;
    T tdiff[3], tmix[3], adv[3];
    T pf[MARCH_PF];
};

template <typename T, int D>
__host__ __device__ __forceinline__ void march_thread(const MarchGeo<D>& G, int tid, MarchThr<T, D>& t)
{
    t.active = tid < G.nact;
    const int tt = t.active ? tid : 0;
    t.x[0] = tt & (G.T[0] - 1);
    t.x[1] = (tt / G.T[0]) & (G.T[1] - 1);
    t.x[2] = tt / (G.T[0] * G.T[1]);
    for (int k = 0; k < 3; ++k) t.j[k] = G.o[k] + t.x[k] + 1;
}

// Coefficient factors of the plane axes (tables as in the streaming operator).  Mem reads tables.
template <typename T, int D, class Mem>
__host__ __device__ __forceinline__ void march_coefs(const MarchGeo<D>& G, const int32_t* utab, const T* tab,
                                                     const T* cst, MarchThr<T, D>& t, Mem& m)
{
    T tphi[3];
    for (int k = 0; k < 3; ++k) {
        t.tdiff[k] = T(0);
        t.tmix[k] = T(0);
        t.adv[k] = T(0);
        tphi[k] = T(0);
    }
    for (int k = 0; k < D - 1; ++k) {
        const T* tk = tab + utab[k];
        const int Mk = G.M[k], jk = t.j[k];
        t.tdiff[k] = m.tab(tk, jk - 1);
        t.tmix[k] = m.tab(tk, Mk + jk - 1);
        tphi[k] = m.tab(tk, 2 * Mk + jk - 1);
    }
    // advection of paper axes 2..N-1 (plane axes 1..d-2), zero on the upper face
    for (int k = 1; k < D - 1; ++k) {
        if (t.j[k] == G.M[k]) continue;
        T s = T(0);
        for (int jj = 1; jj <= k; ++jj) s += m.tab(cst, CST_RHO + k * MAXD + jj) * tphi[jj];
        t.adv[k] = t.tmix[k] * s;
    }
}

// Global -> registers: this thread's share of the slot of plane jv (0 and values beyond the unit's
// lower faces or upper faces read as 0; plane 0 is the lower face).  OP_STAGE2 stages X0 + a X1.
template <typename T, int D, int OP, class Mem>
__host__ __device__ __forceinline__ void march_fetch(const MarchGeo<D>& G, int tid, int jv, const T* X0, const T* X1,
                                                     T a, MarchThr<T, D>& t, Mem& m)
{
    const bool vok = jv >= 1 && jv <= G.M[D - 1];
    const int64_t vb = G.off + (int64_t)(jv - 1) * G.E[D - 1];
#pragma unroll
    for (int r = 0; r < MARCH_PF; ++r) {
        const int e = tid + r * MARCH_THREADS;
        T v = T(0);
        if (e < G.LP && vok) {
            const int y0 = e % G.H[0], y1 = (e / G.H[0]) % G.H[1], y2 = e / G.S2;
            const int y[3] = {y0, y1, y2};
            bool ok = true;
            int64_t g = vb;
            for (int k = 0; k < D - 1; ++k) {
                const int jj = G.o[k] + y[k];            // 1-based: y = 0 is the halo before the tile
                ok = ok && jj >= 1 && jj <= G.M[k];
                g += (int64_t)(jj - 1) * G.E[k];
            }
            if (ok) {
                v = m.ld(X0, g);
                if constexpr (OP == OP_STAGE2) v += a * m.ld(X1, g);
            }
        }
        t.pf[r] = v;
    }
}

// Registers -> the LDS slot of plane jv.
template <typename T, int D, class Mem>
__host__ __device__ __forceinline__ void march_stash(const MarchGeo<D>& G, int tid, int jv, const MarchThr<T, D>& t,
                                                     Mem& m)
{
    const int base = (jv & (MARCH_SLOTS - 1)) * G.LP;
#pragma unroll
    for (int r = 0; r < MARCH_PF; ++r) {
        const int e = tid + r * MARCH_THREADS;
        if (e < G.LP) m.sw(base + e, t.pf[r]);
    }
}

// Sketch 1 with zero lower faces at this thread's node of plane jv, from the LDS slots of planes
// jv - 1, jv, jv + 1: second differences (Neumann ghost on the upper faces), mixed differences for
// every pair (zero on either upper face), advection on the plane axes 1..d-2.  Returns vsq * acc,
// i.e. F before the stage combination; 0 on a Dirichlet rate face (eq bound1_0).  c0 receives the
// node's own value.
template <typename T, int D, class Mem>
__host__ __device__ __forceinline__ T march_F(const MarchGeo<D>& G, const MarchThr<T, D>& t, int jv, const T* tV,
                                              const T* cst, int dirichlet, T& c0, Mem& m)
{
    const int sm = ((jv - 1) & (MARCH_SLOTS - 1)) * G.LP, sc = (jv & (MARCH_SLOTS - 1)) * G.LP,
              sp = ((jv + 1) & (MARCH_SLOTS - 1)) * G.LP;
    const int MV = G.M[D - 1];
    const int S[3] = {1, G.S1, G.S2};
    int c = 0;
    for (int k = 0; k < D - 1; ++k) c += (t.x[k] + 1) * S[k];
    c0 = m.sr(sc + c);
    const bool vtop = jv == MV;
    const T vm = m.sr(sm + c);
    const T vp = vtop ? vm : m.sr(sp + c);
    T acc = m.tab(tV, MV) * (vp - T(2) * c0 + vm);
    const T tmixV = m.tab(tV, MV + 1);
    bool face = false;
    for (int i = 0; i < D - 1; ++i) {
        const bool top = t.j[i] == G.M[i];
        face = face || (dirichlet && top);
        const T xm = m.sr(sc + c - S[i]);
        const T xp = top ? xm : m.sr(sc + c + S[i]);
        acc += t.tdiff[i] * (xp - T(2) * c0 + xm);
        if (i >= 1 && !top) acc += t.adv[i] * (xp - xm);
        // mixed (i, k) with another plane axis k > i
        for (int k = i + 1; k < D - 1; ++k) {
            if (top || t.j[k] == G.M[k]) continue;
            const T xx = m.sr(sc + c + S[i] + S[k]) + m.sr(sc + c - S[i] - S[k]) -
                         m.sr(sc + c + S[i] - S[k]) - m.sr(sc + c - S[i] + S[k]);
            acc += m.tab(cst, CST_RHO + i * MAXD + k) * t.tmix[i] * t.tmix[k] * xx;
        }
        // mixed (i, V)
        if (!top && !vtop) {
            const T xx = m.sr(sp + c + S[i]) + m.sr(sm + c - S[i]) - m.sr(sm + c + S[i]) - m.sr(sp + c - S[i]);
            acc += m.tab(cst, CST_SPHI + i) * t.tmix[i] * tmixV * xx;
        }
    }
    return face ? T(0) : m.tab(tV, jv - 1) * acc;
}

// Global index of this thread's node in plane jv.
template <int D, typename TT>
__host__ __device__ __forceinline__ int64_t march_index(const MarchGeo<D>& G, const TT& t, int jv)
{
    int64_t g = G.off + (int64_t)(jv - 1) * G.E[D - 1];
    for (int k = 0; k < D - 1; ++k) g += (int64_t)(t.j[k] - 1) * G.E[k];
    return g;
}

}  // namespace amf
