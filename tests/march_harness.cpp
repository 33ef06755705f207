// Host emulation of the plane-tiled operator (paper_2408_00559_amd/csrc/amfrw_march.h) for checking
// a plan's blocks before they run on a GPU.  It executes the same phase functions the gfx950 kernel
// executes, thread by thread between the kernel's barriers, with accessors that check
//   - every global read and write lies inside the block's own unit (and the vector),
//   - every coefficient-table read lies inside the table block it indexes,
//   - every LDS index lies inside the block's slot ring, no LDS element is read before it was
//     written, and no element written by one thread is read or written by another thread without a
//     barrier in between,
// and it counts the writes of every node: each inner node of each unit must be written exactly once.
// Built by tests/test_march_harness.py with g++ and loaded through ctypes.
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "amfrw_march.h"

using namespace amf;

namespace {

struct Err {
    std::string msg;
    bool set = false;
    void operator()(const std::string& m)
    {
        if (!set) {
            msg = m;
            set = true;
        }
    }
};

// Coefficient tables of one unit: one block per axis (3 M_i entries for a rate axis, M_V + 2 for V)
// and the per-problem constant block; the emulation allocates them per unit with these sizes.
struct Tables {
    std::vector<double> data;
    std::vector<int32_t> start, size;   // per block
};

struct CheckedMem {
    Err* err;
    int64_t lo = 0, hi = 0;          // the unit's element range
    int64_t total = 0;
    const Tables* tb = nullptr;
    // LDS ring with hazard tracking
    std::vector<double> lds;
    std::vector<int64_t> w_epoch, r_epoch;
    std::vector<int> w_tid, r_tid;   // r_tid: -2 = several readers in r_epoch
    int64_t epoch = 0;
    int tid = 0;
    int64_t reads = 0;

    void reset_lds(int n)
    {
        lds.assign((size_t)n, 0.0);
        w_epoch.assign((size_t)n, -1);
        r_epoch.assign((size_t)n, -1);
        w_tid.assign((size_t)n, -1);
        r_tid.assign((size_t)n, -1);
    }
    double ld(const double* p, int64_t i)
    {
        if (i < lo || i >= hi || i < 0 || i >= total)
            (*err)("global read outside the unit: index " + std::to_string(i) + " not in [" + std::to_string(lo) +
                   ", " + std::to_string(hi) + ")");
        if (i < 0 || i >= total) return 0.0;
        return p[i];
    }
    // one V plane of the unit inside a grid vector (the kernel's buffer resource): a fetch beyond it
    // reads 0 on the GPU, which only the zero elements (MARCH_NONE) and plane 0 (length 0) may rely on
    struct Plane {
        const double* p;
        int64_t base, n;
    };
    Plane plane(const double* p, int64_t base, int64_t n)
    {
        if (n < 0 || (n > 0 && (base < lo || base + n > hi)))
            (*err)("plane range outside the unit: [" + std::to_string(base) + ", +" + std::to_string(n) + ")");
        return {p, base, n};
    }
    double pld(const Plane& h, uint32_t b)
    {
        if (b == MARCH_NONE || h.n == 0) return 0.0;
        if (b % sizeof(double) != 0) (*err)("misaligned byte offset " + std::to_string(b));
        const int64_t i = (int64_t)(b / sizeof(double));
        if (i >= h.n) {
            (*err)("fetch beyond its plane: element " + std::to_string(i) + " of " + std::to_string(h.n));
            return 0.0;
        }
        return ld(h.p, h.base + i);
    }
    double tab(const double* p, int i)
    {
        // find the table block p points into
        const double* base = tb->data.data();
        const int64_t at = p - base;
        for (size_t b = 0; b < tb->start.size(); ++b)
            if (at == tb->start[b]) {
                if (i < 0 || i >= tb->size[b])
                    (*err)("table read outside its block: index " + std::to_string(i) + " of " +
                           std::to_string(tb->size[b]));
                return (i >= 0 && i < tb->size[b]) ? p[i] : 0.0;
            }
        (*err)("table pointer not at a block start");
        return 0.0;
    }
    double sr(int i)
    {
        ++reads;
        if (i < 0 || i >= (int)lds.size()) {
            (*err)("LDS read outside the slot ring: " + std::to_string(i) + " of " + std::to_string(lds.size()));
            return 0.0;
        }
        if (w_epoch[(size_t)i] < 0) (*err)("LDS read before any write at " + std::to_string(i));
        if (w_epoch[(size_t)i] == epoch && w_tid[(size_t)i] != tid)
            (*err)("LDS race: read of " + std::to_string(i) + " written by another thread since the last barrier");
        if (r_epoch[(size_t)i] == epoch) {
            if (r_tid[(size_t)i] != tid) r_tid[(size_t)i] = -2;
        } else {
            r_epoch[(size_t)i] = epoch;
            r_tid[(size_t)i] = tid;
        }
        return lds[(size_t)i];
    }
    void sw(int i, double v)
    {
        if (i < 0 || i >= (int)lds.size()) {
            (*err)("LDS write outside the slot ring: " + std::to_string(i) + " of " + std::to_string(lds.size()));
            return;
        }
        if (w_epoch[(size_t)i] == epoch && w_tid[(size_t)i] != tid)
            (*err)("LDS race: two threads write " + std::to_string(i) + " between barriers");
        if (r_epoch[(size_t)i] == epoch && r_tid[(size_t)i] != tid)
            (*err)("LDS race: write of " + std::to_string(i) + " read by another thread since the last barrier");
        w_epoch[(size_t)i] = epoch;
        w_tid[(size_t)i] = tid;
        lds[(size_t)i] = v;
    }
};

// One block in the kernel's order: V^2 factors into LDS, planes v0 .. v0 + 2 fetched and stashed,
// planes v0 + 3 .. v0 + 2 + MARCH_DEPTH fetched (register set i mod MARCH_DEPTH for plane v0 + i), the
// first node's stage values loaded, barrier, the crosses of planes v0 and v0 + 1 read; per step stash
// plane jv + 2, fetch plane jv + 2 + MARCH_DEPTH into the same registers (an empty range past the
// block's last plane), load the next node's stage values (an empty range on the last step), read the
// cross of plane jv + 1 (not on the V face), compute and store plane jv, barrier.
template <int D, int OP, class Sh>
void walk_block(const MarchBlk& B, const int8_t* ul, int64_t uoff, int64_t total, CheckedMem& m, std::vector<double>& X0,
                std::vector<double>& X1, std::vector<double>& cG, std::vector<double>& X2, std::vector<double>& W,
                std::vector<double>& Sv, bool fuse, int32_t* writes, Err& err)
{
    constexpr int NPF = Sh::NPF;
    // the unit's tables: blocks per axis, then the constant block
    Tables tb;
    int32_t at = 0;
    int32_t utab[MAXD] = {};
    for (int i = 0; i < D; ++i) {
        const int M = 1 << ul[i];
        const int sz = i < D - 1 ? 3 * M : M + 2;
        utab[i] = at;
        tb.start.push_back(at);
        tb.size.push_back(sz);
        at += sz;
    }
    const int32_t cst0 = at;
    tb.start.push_back(at);
    tb.size.push_back(CST_SIZE);
    at += CST_SIZE;
    tb.data.assign((size_t)at, 0.01);
    m.tb = &tb;
    MarchGeo<D> G;
    march_geo<D>(ul, uoff, B, G);
    {
        const int lt[3] = {B.lt[0], B.lt[1], B.lt[2]};
        if (G.LP > MARCH_MAX_PLANE || G.LP != march_slot_elems(D, lt)) {
            err("plane slot larger than MARCH_MAX_PLANE or sized differently from the host");
            return;
        }
        if (B.shape != march_shape_id(D, lt)) {
            err("block shape index differs from its tile");
            return;
        }
    }
    if (G.nact > MARCH_THREADS) {
        err("tile has more nodes than threads");
        return;
    }
    if (Sh::FULL && (G.nact != MARCH_THREADS || Sh::t0(G) != G.T[0] || Sh::t1(G) != G.T[1] || Sh::s1(G) != G.S1 ||
                     Sh::s2(G) != G.S2 || Sh::lp(G) != G.LP)) {
        err("compiled stride set differs from the block's tile");
        return;
    }
    if (!Sh::FULL && NPF * MARCH_THREADS < G.LP) {
        err("prefetch registers do not cover the slot");
        return;
    }
    m.reset_lds(MARCH_SLOTS * G.LP + MARCH_SEG);   // slot ring + V^2 words (sized for the plan's largest slot)
    const double* tab = tb.data.data();
    const double* cst = tab + cst0;
    std::vector<MarchThr<double, D, NPF>> thr(MARCH_THREADS);
    for (int t = 0; t < MARCH_THREADS; ++t) {
        m.tid = t;
        march_thread<double, D, Sh>(G, t, thr[(size_t)t]);
        march_coefs<double, D>(G, utab, tab, cst, thr[(size_t)t], m);
        march_face<double, D>(0, thr[(size_t)t]);
    }
    const int MV = G.M[D - 1];
    const int last = std::min(MV, G.v0 + G.vn + 1);
    const double* cE = OP == OP_REFINE ? W.data() : cG.data();
    auto centre = [&](int t, int jv, bool live) {
        const MarchThr<double, D, NPF>& th = thr[(size_t)t];
        const int64_t b = march_plane_base<D>(G, jv), n = live ? march_plane_len<D>(G, jv) : 0;
        const double e0 = m.pld(m.plane(cE, b, n), th.gob);
        const double e1 = OP == OP_STAGE2 ? m.pld(m.plane(X2.data(), b, n), th.gob) : 0.0;
        return std::make_pair(e0, e1);
    };
    const double* tV = tab + utab[D - 1];
    std::vector<std::pair<double, double>> cur((size_t)MARCH_THREADS), nxt((size_t)MARCH_THREADS);
    constexpr int DP = MARCH_DEPTH;
    std::vector<std::array<MarchPf<double, OP, NPF>, DP>> pf((size_t)MARCH_THREADS);
    for (int t = 0; t < MARCH_THREADS; ++t) {
        m.tid = t;
        march_vsq<double, D, Sh>(G, t, tV, m);
        for (int i = 0; i < 3 + DP; ++i) {
            const int p = G.v0 + i;
            if (i >= DP && p - DP <= last)
                march_stash<double, D, Sh>(G, t, p - DP, pf[(size_t)t][(size_t)((i - DP) % DP)], 0.5, m);
            march_fetch<double, D, OP>(G, p, X0.data(), X1.data(), thr[(size_t)t], pf[(size_t)t][(size_t)(i % DP)], m,
                                       p <= last);
        }
        cur[(size_t)t] = centre(t, G.v0 + 1, true);
    }
    ++m.epoch;                                               // __syncthreads
    // crosses of planes v0 and v0 + 1, then each step the cross of plane jv + 1 (register window)
    constexpr int NX = MarchX<D>::N;
    std::vector<std::array<std::array<double, NX>, 3>> win((size_t)MARCH_THREADS);
    auto cross = [&](int t, int jv, int slot) {
        double x[NX];
        march_cross<double, D, Sh>(G, thr[(size_t)t], jv, x, m);
        for (int k = 0; k < NX; ++k) win[(size_t)t][(size_t)slot][(size_t)k] = x[k];
    };
    for (int t = 0; t < MARCH_THREADS; ++t) {
        m.tid = t;
        if (!thr[(size_t)t].active) continue;
        cross(t, G.v0, 0);
        cross(t, G.v0 + 1, 1);
    }
    for (int s = 1; s <= G.vn && !err.set; ++s) {
        const int jv = G.v0 + s;
        const int im = (s - 1) % 3, ic = s % 3, ip = (s + 1) % 3;
        for (int t = 0; t < MARCH_THREADS; ++t) {
            m.tid = t;
            MarchThr<double, D, NPF>& th = thr[(size_t)t];
            MarchPf<double, OP, NPF>& q = pf[(size_t)t][(size_t)(((s - 1) + 1) % DP)];   // holds plane jv + 2
            if (jv + 2 <= last) march_stash<double, D, Sh>(G, t, jv + 2, q, 0.5, m);
            march_fetch<double, D, OP>(G, jv + 2 + DP, X0.data(), X1.data(), th, q, m, jv + 2 + DP <= last);
            nxt[(size_t)t] = centre(t, jv + 1, s < G.vn);
            const double vsq = march_vsq_of<double, D, Sh>(G, s, m);
            if (th.active) {
                if (jv < MV) cross(t, jv + 1, ip);
                double xm[NX], xc[NX], xp[NX];
                for (int k = 0; k < NX; ++k) {
                    xm[k] = win[(size_t)t][(size_t)im][(size_t)k];
                    xc[k] = win[(size_t)t][(size_t)ic][(size_t)k];
                    xp[k] = jv < MV ? win[(size_t)t][(size_t)ip][(size_t)k] : std::nan("");
                }
                const double F = march_F<double, D, Sh>(G, th, jv, vsq, m.tab(tV, MV), xm, xc, xp, m);
                if (F != F) err("the operator used the cross of the plane beyond the V face");
                const double c0 = xc[0];
                const double e0 = cur[(size_t)t].first, e1 = cur[(size_t)t].second;
                double o;
                if (OP == OP_STAGE1) o = 0.1 * (F + e0);
                else if (OP == OP_STAGE2) o = 0.1 * (F + e0) + 0.3 * e1;
                else o = 2.0 * e0 - c0 + 0.1 * F;
                // fused axis-1 solve: the row's factors lie inside the unit's factor block (M_V planes
                // of 3 M_1 entries); the refinement then stores only the solved value
                const bool fz = march_fused<D>(G, fuse);
                if (fz) {
                    const int fa = march_fac_at<double, D>(G, jv, th);
                    const int fsize = 3 * G.M[0] * G.M[D - 1];
                    if (G.T[0] != G.M[0] || G.o[0] != 0) err("fused block whose tile row is not a whole axis-1 line");
                    for (int q = 0; q < 3; ++q)
                        if (fa + q * G.M[0] < 0 || fa + q * G.M[0] >= fsize) err("factor read outside the unit's block");
                }
                auto store = [&](std::vector<double>& V, bool count) {
                    const CheckedMem::Plane hw = m.plane(V.data(), march_plane_base<D>(G, jv), march_plane_len<D>(G, jv));
                    if (hw.n == 0 || th.gob % sizeof(double) != 0 || (int64_t)(th.gob / sizeof(double)) >= hw.n) {
                        err("store outside its plane");
                        return;
                    }
                    const int64_t g = hw.base + (int64_t)(th.gob / sizeof(double));
                    if (g < m.lo || g >= m.hi) err("global write outside the unit");
                    if (g >= 0 && g < total) {
                        V[(size_t)g] = o;
                        if (count) writes[g] += 1;
                    }
                };
                if (!(fz && OP == OP_REFINE)) store(W, true);
                if (fz) store(Sv, OP == OP_REFINE);
            }
            cur[(size_t)t] = nxt[(size_t)t];
        }
        ++m.epoch;                                           // __syncthreads
    }
}

template <int D, int OP>
int run(int n_units, const int8_t* lv, const int64_t* off, int64_t total, int elem, bool xorder, bool fuse,
        int64_t blk_first, int64_t blk_stride, int64_t* n_blocks_out, int64_t* lds_reads_out, int32_t* writes, Err& err)
{
    std::vector<MarchBlk> blocks;
    march_blocks(D, n_units, lv, MAXD, elem, blocks);
    *n_blocks_out = (int64_t)blocks.size();
    if (xorder) {                                    // the table the kernel reads when xcd != 0
        std::vector<MarchBlk> ordered;
        march_order_xcd(blocks, 8, ordered);
        if (ordered.size() % 8 != 0) {
            err("XCD-ordered table is not a whole number of rounds");
            return 1;
        }
        blocks.swap(ordered);
    }
    std::vector<double> X0((size_t)total, 0.5), X1((size_t)total, 0.25), cG((size_t)total, 0.125),
        X2((size_t)total, 1.0), W((size_t)total, 0.0), Sv((size_t)total, 0.0);
    CheckedMem m;
    m.err = &err;
    m.total = total;
    for (int64_t bi = blk_first; bi < (int64_t)blocks.size() && !err.set; bi += blk_stride) {
        const MarchBlk& B = blocks[(size_t)bi];
        if (B.vn == 0) continue;                     // padding: the kernel returns at once
        const int u = B.unit;
        if (u < 0 || u >= n_units) {
            err("block names a unit out of range");
            break;
        }
        const int8_t* ul = lv + (size_t)u * MAXD;
        int lsum = 0;
        for (int i = 0; i < D; ++i) lsum += ul[i];
        m.lo = off[u];
        m.hi = off[u] + ((int64_t)1 << lsum);
        march_dispatch<D>(B.shape, [&](auto sh) {
            walk_block<D, OP, decltype(sh)>(B, ul, off[u], total, m, X0, X1, cG, X2, W, Sv, fuse, writes, err);
        });
    }
    *lds_reads_out = m.reads;
    return err.set ? 1 : 0;
}

template <int D>
int run_op(int op, int n_units, const int8_t* lv, const int64_t* off, int64_t total, int elem, bool xorder, bool fuse,
           int64_t first, int64_t stride, int64_t* nb, int64_t* reads, int32_t* writes, Err& err)
{
    if (op == OP_STAGE1)
        return run<D, OP_STAGE1>(n_units, lv, off, total, elem, xorder, fuse, first, stride, nb, reads, writes, err);
    if (op == OP_STAGE2)
        return run<D, OP_STAGE2>(n_units, lv, off, total, elem, xorder, fuse, first, stride, nb, reads, writes, err);
    return run<D, OP_REFINE>(n_units, lv, off, total, elem, xorder, fuse, first, stride, nb, reads, writes, err);
}

}  // namespace

extern "C" {

// Walk entries first, first + stride, ... of the plan's marching-operator block table (every entry
// for stride 1): the unit-by-unit table, or with xorder the XCD-grouped one; fuse: the operator also
// solves the axis-1 lines of the units whose lines fit one tile row.  lv: [n_units][MAXD]
// levels; off: unit offsets; writes: [total] counters (incremented).  Returns 0 when every check
// passed, else 1 with the first failure in err.
int march_check(int d, int op, int n_units, const int8_t* lv, const int64_t* off, int64_t total, int elem, int xorder,
                int fuse, int64_t first, int64_t stride, int64_t* n_blocks, int64_t* lds_reads, int32_t* writes,
                char* err, int errlen)
{
    Err e;
    int rc = 2;
    const bool xo = xorder != 0, fz = fuse != 0;
    if (d == 2) rc = run_op<2>(op, n_units, lv, off, total, elem, xo, fz, first, stride, n_blocks, lds_reads, writes, e);
    else if (d == 3) rc = run_op<3>(op, n_units, lv, off, total, elem, xo, fz, first, stride, n_blocks, lds_reads, writes, e);
    else if (d == 4) rc = run_op<4>(op, n_units, lv, off, total, elem, xo, fz, first, stride, n_blocks, lds_reads, writes, e);
    else e("d must lie in [2, 4]");
    std::snprintf(err, (size_t)errlen, "%s", e.msg.c_str());
    return e.set ? 1 : rc;
}

int march_maxd(void) { return MAXD; }

}  // extern "C"
