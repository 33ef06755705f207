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

template <int D, int OP>
int run(int n_units, const int8_t* lv, const int64_t* off, int64_t total, int elem, bool deep, bool xorder,
        int64_t blk_first, int64_t blk_stride, int64_t* n_blocks_out, int64_t* lds_reads_out, int32_t* writes,
        Err& err)
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
    const bool ahead = OP != OP_STAGE2;              // stage values loaded one plane ahead
    std::vector<double> X0((size_t)total, 0.5), X1((size_t)total, 0.25), cG((size_t)total, 0.125),
        X2((size_t)total, 1.0), W((size_t)total, 0.0);
    CheckedMem m;
    m.err = &err;
    m.total = total;
    std::vector<MarchThr<double, D>> thr(MARCH_THREADS);
    int64_t reads = 0;
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
        march_geo<D>(ul, off[u], B, G);
        {
            const int lt[3] = {B.lt[0], B.lt[1], B.lt[2]};
            if (G.SLOT > MARCH_MAX_PLANE || G.SLOT != march_slot_elems(D, lt, B.h0)) {
                err("plane slot larger than MARCH_MAX_PLANE or sized differently from the host");
                break;
            }
        }
        if (G.nact > MARCH_THREADS) {
            err("tile has more nodes than threads");
            break;
        }
        m.reset_lds(MARCH_SLOTS * G.SLOT);      // the kernel's dynamic LDS is sized for the plan's largest slot
        const double* tab = tb.data.data();
        const double* cst = tab + cst0;
        for (int t = 0; t < MARCH_THREADS; ++t) {
            m.tid = t;
            march_thread<double, D>(G, t, thr[(size_t)t]);
            march_coefs<double, D>(G, utab, tab, cst, thr[(size_t)t], m);
            march_face<double, D>(0, thr[(size_t)t]);
            march_pads<double, D>(G, t, m);
        }
        const int MV = G.M[D - 1];
        const int last = std::min(MV, G.v0 + G.vn + 1);
        // the kernel's order: planes v0 .. v0 + 2 fetched and stashed, then (deep pipeline) plane
        // v0 + 3 fetched, the first node's stage values loaded (all but stage 2), barrier; per step
        // (deep) stash plane jv + 2 and fetch jv + 3, or (one plane) fetch jv + 2; load the next
        // node's stage values; compute and store plane jv; (one plane) stash plane jv + 2; barrier
        auto centre = [&](int t, int jv) {
            const MarchThr<double, D>& th = thr[(size_t)t];
            const int64_t g = th.active ? march_index<D>(G, th, jv) : G.off;
            if (OP == OP_REFINE) return std::make_pair(m.ld(W.data(), g), 0.0);
            return std::make_pair(m.ld(cG.data(), g), OP == OP_STAGE2 ? m.ld(X2.data(), g) : 0.0);
        };
        std::vector<std::pair<double, double>> cur((size_t)MARCH_THREADS), nxt((size_t)MARCH_THREADS);
        for (int t = 0; t < MARCH_THREADS; ++t) {
            m.tid = t;
            for (int p = G.v0; p <= G.v0 + 2 && p <= last; ++p) {
                march_fetch<double, D, OP>(G, p, X0.data(), X1.data(), 0.5, thr[(size_t)t], m);
                march_stash<double, D>(G, t, p, thr[(size_t)t], m);
            }
            if (deep && G.v0 + 3 <= last)
                march_fetch<double, D, OP>(G, G.v0 + 3, X0.data(), X1.data(), 0.5, thr[(size_t)t], m);
            cur[(size_t)t] = ahead ? centre(t, G.v0 + 1) : std::make_pair(0.0, 0.0);
        }
        ++m.epoch;                                           // __syncthreads
        const double* tV = tab + utab[D - 1];
        for (int s = 1; s <= G.vn && !err.set; ++s) {
            const int jv = G.v0 + s;
            for (int t = 0; t < MARCH_THREADS; ++t) {
                m.tid = t;
                MarchThr<double, D>& th = thr[(size_t)t];
                if (deep) {
                    if (jv + 2 <= last) march_stash<double, D>(G, t, jv + 2, th, m);
                    if (jv + 3 <= last) march_fetch<double, D, OP>(G, jv + 3, X0.data(), X1.data(), 0.5, th, m);
                } else if (jv + 2 <= last) {
                    march_fetch<double, D, OP>(G, jv + 2, X0.data(), X1.data(), 0.5, th, m);
                }
                nxt[(size_t)t] = ahead && s < G.vn ? centre(t, jv + 1) : std::make_pair(0.0, 0.0);
                const double vsq = m.tab(tV, jv - 1);
                if (th.active) {
                    double c0;
                    const double F = march_F<double, D>(G, th, jv, vsq, m.tab(tV, MV), c0, m);
                    const int64_t g = march_index<D>(G, th, jv);
                    if (!ahead) cur[(size_t)t] = centre(t, jv);
                    const double e0 = cur[(size_t)t].first, e1 = cur[(size_t)t].second;
                    double o;
                    if (OP == OP_STAGE1) o = 0.1 * (F + e0);
                    else if (OP == OP_STAGE2) o = 0.1 * (F + e0) + 0.3 * e1;
                    else o = 2.0 * e0 - c0 + 0.1 * F;
                    if (g < m.lo || g >= m.hi) err("global write outside the unit");
                    if (g >= 0 && g < total) {
                        W[(size_t)g] = o;
                        writes[g] += 1;
                    }
                }
                if (ahead) cur[(size_t)t] = nxt[(size_t)t];
                if (!deep && jv + 2 <= last) march_stash<double, D>(G, t, jv + 2, th, m);
            }
            ++m.epoch;                                       // __syncthreads
        }
    }
    reads += m.reads;
    *lds_reads_out = reads;
    return err.set ? 1 : 0;
}

template <int D>
int run_op(int op, int n_units, const int8_t* lv, const int64_t* off, int64_t total, int elem, bool deep, bool xorder,
           int64_t first, int64_t stride, int64_t* nb, int64_t* reads, int32_t* writes, Err& err)
{
    if (op == OP_STAGE1)
        return run<D, OP_STAGE1>(n_units, lv, off, total, elem, deep, xorder, first, stride, nb, reads, writes, err);
    if (op == OP_STAGE2)
        return run<D, OP_STAGE2>(n_units, lv, off, total, elem, deep, xorder, first, stride, nb, reads, writes, err);
    return run<D, OP_REFINE>(n_units, lv, off, total, elem, deep, xorder, first, stride, nb, reads, writes, err);
}

}  // namespace

extern "C" {

// Walk entries first, first + stride, ... of the plan's marching-operator block table (every entry
// for stride 1): the unit-by-unit table, or with xorder the XCD-grouped one; deep selects the
// two-plane pipeline.  lv: [n_units][MAXD] levels; off: unit offsets; writes: [total] counters
// (incremented).  Returns 0 when every check passed, else 1 with the first failure in err.
int march_check(int d, int op, int n_units, const int8_t* lv, const int64_t* off, int64_t total, int elem, int deep,
                int xorder, int64_t first, int64_t stride, int64_t* n_blocks, int64_t* lds_reads, int32_t* writes,
                char* err, int errlen)
{
    Err e;
    int rc = 2;
    const bool dp = deep != 0, xo = xorder != 0;
    if (d == 2) rc = run_op<2>(op, n_units, lv, off, total, elem, dp, xo, first, stride, n_blocks, lds_reads, writes, e);
    else if (d == 3)
        rc = run_op<3>(op, n_units, lv, off, total, elem, dp, xo, first, stride, n_blocks, lds_reads, writes, e);
    else if (d == 4)
        rc = run_op<4>(op, n_units, lv, off, total, elem, dp, xo, first, stride, n_blocks, lds_reads, writes, e);
    else e("d must lie in [2, 4]");
    std::snprintf(err, (size_t)errlen, "%s", e.msg.c_str());
    return e.set ? 1 : rc;
}

int march_maxd(void) { return MAXD; }

}  // extern "C"
