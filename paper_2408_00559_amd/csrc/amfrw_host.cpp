// Host side of libamfrw: descriptor validation, enumeration of the combination technique's
// component grids, 1-D coefficient tables, workspace layout and the C ABI of include/amfrw.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "amfrw.h"
#include "amfrw_internal.h"

using namespace amf;

namespace {

thread_local std::string g_err;

amf_status fail(amf_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

amf_status hip_fail(hipError_t e, const char* what)
{
    return fail(AMF_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr int RHO_LD = AMF_MAX_D - 1;   // leading dimension of amf_problem::rho

}  // namespace

enum VecId { V_Y = 0, V_K1 = 1, V_A = 2, V_B = 3, V_C = 4, N_VEC = 5 };

struct amf_plan {
    int d = 0, prec = 0, steps = 0, richardson = 0, n_probs = 0, n_units = 0;
    amf_scheme sch{};
    std::vector<amf_problem> probs;
    std::vector<UnitDev> units;            // n_units + sentinel
    std::vector<double> coef;              // combination coefficient per unit
    std::vector<double> tabd;              // coefficient tables in FP64
    std::vector<ProbDev> probdev;
    std::vector<int32_t> blk_unit;
    std::vector<int32_t> ax_units[MAXD];
    std::vector<int64_t> ax_line_off[MAXD];
    std::vector<SweepBlk> ax_blk[MAXD];
    int64_t total = 0;

    size_t off_vec[N_VEC]{}, off_units = 0, off_probs = 0, off_tab = 0, off_blk = 0;
    size_t off_axu[MAXD]{}, off_axl[MAXD]{}, off_axb[MAXD]{};
    size_t off_coef = 0, off_vals = 0, off_valsc = 0, ws_bytes = 0;
    size_t elem = 8;

    char* ws = nullptr;
    bool bound = false, initialised = false, have_coarse = false;
    DevPlan dev{};

    // per-kernel event timing
    struct ProfRec {
        int kclass;
        hipEvent_t a, b;
        double bytes;
    };
    bool prof = false;
    std::vector<hipEvent_t> pool;
    size_t pool_next = 0;
    std::vector<ProfRec> recs;

    void* vec(int v) const { return ws + off_vec[v]; }
    double vbytes() const { return (double)total * (double)elem; }

    ~amf_plan()
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

namespace {

// Grids of the combination technique: q = 0..d-1, every l with |l|_1 = n - q (levels psi + l_i),
// coefficient (-1)^q C(d-1, q); q ascending, then lexicographic with the last entry fastest.
void enumerate_grids(int d, int n, int psi, std::vector<std::vector<int>>& lv, std::vector<double>& cf)
{
    for (int q = 0; q < d; ++q) {
        const int target = n - q;
        if (target < 0) continue;
        double binom = 1.0;
        for (int i = 1; i <= q; ++i) binom = binom * (double)(d - 1 - q + i) / (double)i;
        const double c = (q % 2 ? -1.0 : 1.0) * binom;
        std::vector<int> l(d, 0);
        // recursive odometer over the first d-1 entries
        for (;;) {
            int s = 0;
            for (int i = 0; i < d - 1; ++i) s += l[i];
            if (s <= target) {
                std::vector<int> row(d);
                for (int i = 0; i < d - 1; ++i) row[i] = psi + l[i];
                row[d - 1] = psi + target - s;
                lv.push_back(row);
                cf.push_back(c);
            }
            int pos = d - 2;
            while (pos >= 0 && ++l[pos] > target) l[pos--] = 0;
            if (pos < 0) break;
        }
    }
}

amf_status validate_problem(const amf_problem& p, int d, int idx)
{
    const std::string at = " (problem " + std::to_string(idx) + ")";
    if (p.struct_size != sizeof(amf_problem)) return fail(AMF_E_INVALID, "amf_problem.struct_size mismatch" + at);
    if (p.d != d) return fail(AMF_E_INVALID, "all problems must share d" + at);
    if (p.payoff != AMF_PAYOFF_CAPLET && p.payoff != AMF_PAYOFF_SWAPTION)
        return fail(AMF_E_INVALID, "unknown payoff" + at);
    if (!(p.beta >= 0.0 && p.beta <= 1.0)) return fail(AMF_E_INVALID, "beta must lie in [0,1]" + at);
    if (!(p.sigma >= 0.0) || !std::isfinite(p.sigma)) return fail(AMF_E_INVALID, "sigma must be >= 0" + at);
    if (!(p.maturity > 0.0) || !std::isfinite(p.maturity)) return fail(AMF_E_INVALID, "maturity must be > 0" + at);
    if (!std::isfinite(p.strike) || !std::isfinite(p.discount)) return fail(AMF_E_INVALID, "strike/discount not finite" + at);
    for (int i = 0; i < d - 1; ++i) {
        if (!(p.alpha[i] >= 0.0) || !std::isfinite(p.alpha[i])) return fail(AMF_E_INVALID, "alpha must be >= 0" + at);
        if (!(std::fabs(p.phi[i]) <= 1.0)) return fail(AMF_E_INVALID, "|phi| must be <= 1" + at);
        if (!(p.tau[i] >= 0.0) || !std::isfinite(p.tau[i])) return fail(AMF_E_INVALID, "tau must be >= 0" + at);
        for (int k = 0; k < d - 1; ++k) {
            const double r = p.rho[i * RHO_LD + k];
            if (!(std::fabs(r) <= 1.0)) return fail(AMF_E_INVALID, "|rho| must be <= 1" + at);
            if (std::fabs(r - p.rho[k * RHO_LD + i]) > 1e-12) return fail(AMF_E_INVALID, "rho must be symmetric" + at);
        }
        if (p.rho[i * RHO_LD + i] != 1.0) return fail(AMF_E_INVALID, "rho must have a unit diagonal" + at);
    }
    for (int i = 0; i < d; ++i) {
        if (!(p.x_max[i] > 0.0) || !std::isfinite(p.x_max[i])) return fail(AMF_E_INVALID, "x_max must be > 0" + at);
        if (!(p.x_eval[i] >= 0.0 && p.x_eval[i] <= p.x_max[i]))
            return fail(AMF_E_INVALID, "x_eval outside the domain" + at);
    }
    return AMF_OK;
}

// FP64 1-D factors of the coefficients (coef_diff), (coef_mix), (coef_adv) for one axis/level.
void append_axis_table(std::vector<double>& t, const amf_problem& p, int axis, int level)
{
    const int d = p.d;
    const int M = 1 << level;
    const double h = p.x_max[axis] / (double)M;
    if (axis < d - 1) {
        const double a = p.alpha[axis], rii = p.rho[axis * RHO_LD + axis], tau = p.tau[axis];
        const size_t b = t.size();
        t.resize(b + 3 * (size_t)M);
        for (int r = 0; r < M; ++r) {
            const double x = (double)(r + 1) * h;
            const double xb = std::pow(x, p.beta);
            t[b + r] = 0.5 * a * a * rii * std::pow(x, 2.0 * p.beta) / (h * h);      // d_i / (h^2 V^2)
            t[b + M + r] = a * xb / (2.0 * h);                                      // alpha F^beta / 2h
            t[b + 2 * M + r] = a * tau * xb / (1.0 + tau * x);                      // alpha Phi_beta
        }
    } else {
        const size_t b = t.size();
        t.resize(b + (size_t)M + 2);
        for (int r = 0; r < M; ++r) {
            const double v = (double)(r + 1) * h;
            t[b + r] = v * v;                                                       // V^2
        }
        t[b + M] = 0.5 * p.sigma * p.sigma / (h * h);                               // d_N/(h^2 V^2)
        t[b + M + 1] = 1.0 / (2.0 * h);
    }
}

template <typename T>
std::vector<T> cast_vec(const std::vector<double>& v)
{
    std::vector<T> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = (T)v[i];
    return o;
}

amf_status upload(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return AMF_OK;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    return AMF_OK;
}

}  // namespace

extern "C" {

int32_t amf_abi_version(void) { return AMF_ABI_VERSION; }

const char* amf_last_error(void) { return g_err.c_str(); }

amf_status amf_scheme_amfrw2(amf_scheme* out)
{
    if (!out) return fail(AMF_E_INVALID, "null scheme");
    std::memset(out, 0, sizeof(*out));
    out->struct_size = sizeof(amf_scheme);
    out->stages = 2;
    out->a[1 * AMF_MAX_STAGES + 0] = 2.0 / 3.0;
    out->q[1 * AMF_MAX_STAGES + 0] = -4.0 / 3.0;
    out->b[0] = 5.0 / 4.0;
    out->b[1] = 3.0 / 4.0;
    out->theta = (3.0 + std::sqrt(3.0)) / 6.0;
    out->nu = out->theta;
    return AMF_OK;
}

amf_status amf_plan_create(const amf_problem* probs, int32_t n_probs, const amf_grid_spec* grid,
                           const amf_scheme* scheme, amf_precision precision, int32_t n_steps,
                           int32_t richardson, amf_plan** out)
{
    g_err.clear();
    if (!out) return fail(AMF_E_INVALID, "null output pointer");
    *out = nullptr;
    if (!probs || n_probs < 1) return fail(AMF_E_INVALID, "need at least one problem");
    if (!grid || grid->struct_size != sizeof(amf_grid_spec)) return fail(AMF_E_INVALID, "bad amf_grid_spec");
    if (!scheme || scheme->struct_size != sizeof(amf_scheme)) return fail(AMF_E_INVALID, "bad amf_scheme");
    if (precision != AMF_FP64 && precision != AMF_FP32) return fail(AMF_E_INVALID, "unknown precision");
    if (n_steps < 1) return fail(AMF_E_INVALID, "n_steps must be >= 1");
    if (richardson != 0 && richardson != 1) return fail(AMF_E_INVALID, "richardson must be 0 or 1");
    if (scheme->stages != 2) return fail(AMF_E_UNSUPPORTED, "only 2-stage AMFR-W schemes are built");
    if (!(scheme->theta > 0.0) || !(scheme->nu > 0.0)) return fail(AMF_E_INVALID, "theta and nu must be > 0");
    const int d = probs[0].d;
    if (d < 2 || d > MAXD) return fail(AMF_E_INVALID, "d must lie in [2, 6]");
    for (int p = 0; p < n_probs; ++p) {
        amf_status st = validate_problem(probs[p], d, p);
        if (st != AMF_OK) return st;
    }
    std::vector<std::vector<int>> glv;
    std::vector<double> gcf;
    if (grid->full_grid) {
        std::vector<int> row(d);
        int s = 0;
        for (int i = 0; i < d; ++i) {
            if (grid->levels[i] < 0 || grid->levels[i] > 16) return fail(AMF_E_INVALID, "levels must lie in [0, 16]");
            row[i] = grid->levels[i];
            s += row[i];
        }
        if (s > 30) return fail(AMF_E_INVALID, "full grid too large (sum of levels > 30)");
        glv.push_back(row);
        gcf.push_back(1.0);
    } else {
        if (grid->psi < 0 || grid->psi > 8) return fail(AMF_E_INVALID, "psi must lie in [0, 8]");
        if (grid->n < d - 1) return fail(AMF_E_INVALID, "n must be >= d-1");
        if (grid->psi + grid->n > 16 || d * grid->psi + grid->n > 30)
            return fail(AMF_E_INVALID, "combination level too large");
        enumerate_grids(d, grid->n, grid->psi, glv, gcf);
    }

    amf_plan* P = new (std::nothrow) amf_plan();
    if (!P) return fail(AMF_E_NOMEM, "out of host memory");
    try {
        P->d = d;
        P->prec = (int)precision;
        P->elem = precision == AMF_FP64 ? 8 : 4;
        P->steps = n_steps;
        P->richardson = richardson;
        P->n_probs = n_probs;
        P->sch = *scheme;
        P->probs.assign(probs, probs + n_probs);
        const int ng = (int)glv.size();
        const int64_t nu64 = (int64_t)ng * n_probs;
        if (nu64 > (int64_t)1 << 30) {
            delete P;
            return fail(AMF_E_INVALID, "too many units");
        }
        P->n_units = (int)nu64;

        // coefficient tables: per problem a constant block, then (axis, level) blocks
        for (int p = 0; p < n_probs; ++p) {
            const amf_problem& pr = probs[p];
            ProbDev pd{};
            for (int i = 0; i < d; ++i) {
                pd.xmax[i] = pr.x_max[i];
                pd.xeval[i] = pr.x_eval[i];
            }
            for (int i = 0; i < d - 1; ++i) pd.tau[i] = pr.tau[i];
            pd.K = pr.strike;
            pd.discount = pr.discount;
            pd.payoff = pr.payoff;
            pd.cst = (int32_t)P->tabd.size();
            pd.unit_begin = p * ng;
            pd.unit_end = (p + 1) * ng;
            std::vector<double> c(CST_SIZE, 0.0);
            for (int i = 0; i < d - 1; ++i) {
                for (int k = 0; k < d - 1; ++k) c[CST_RHO + i * MAXD + k] = pr.rho[i * RHO_LD + k];
                c[CST_SPHI + i] = pr.sigma * pr.phi[i];
            }
            const double dt = pr.maturity / (double)n_steps;
            for (int run = 0; run < 2; ++run) {
                const double h = run == 0 ? dt : 0.5 * dt;
                c[CST_RUN + 3 * run + 0] = h;
                c[CST_RUN + 3 * run + 1] = scheme->nu * h;
                c[CST_RUN + 3 * run + 2] = scheme->theta * h;
            }
            P->tabd.insert(P->tabd.end(), c.begin(), c.end());
            // axis tables for every level in use on that axis
            std::vector<int32_t> blk_of[MAXD];
            for (int i = 0; i < d; ++i) blk_of[i].assign(17, -1);
            for (int g = 0; g < ng; ++g)
                for (int i = 0; i < d; ++i) {
                    const int L = glv[g][i];
                    if (blk_of[i][L] < 0) {
                        if (P->tabd.size() > (size_t)INT32_MAX / 2) throw std::bad_alloc();
                        blk_of[i][L] = (int32_t)P->tabd.size();
                        append_axis_table(P->tabd, pr, i, L);
                    }
                }
            P->probdev.push_back(pd);
            for (int g = 0; g < ng; ++g) {
                UnitDev U{};
                U.off = P->total;
                U.prob = p;
                int ls = 0;
                for (int i = 0; i < d; ++i) {
                    U.lv[i] = (int8_t)glv[g][i];
                    U.tab[i] = blk_of[i][glv[g][i]];
                    ls += glv[g][i];
                }
                U.lsum = ls;
                P->units.push_back(U);
                P->coef.push_back(gcf[g]);
                P->total += (int64_t)1 << ls;
            }
        }
        UnitDev sentinel{};
        sentinel.off = P->total;
        P->units.push_back(sentinel);

        // node blocks -> first unit
        const int64_t nblk = (P->total + NODE_BLOCK - 1) / NODE_BLOCK;
        P->blk_unit.resize(nblk);
        {
            int u = 0;
            for (int64_t b = 0; b < nblk; ++b) {
                const int64_t g0 = b * NODE_BLOCK;
                while (g0 >= P->units[u + 1].off) ++u;
                P->blk_unit[b] = u;
            }
        }
        // per axis: units ordered by M_axis, line offsets, blocks that never mix line lengths
        for (int ax = 0; ax < d; ++ax) {
            std::vector<int32_t>& ord = P->ax_units[ax];
            ord.resize(P->n_units);
            for (int u = 0; u < P->n_units; ++u) ord[u] = u;
            std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
                return P->units[a].lv[ax] < P->units[b].lv[ax];
            });
            std::vector<int64_t>& lo = P->ax_line_off[ax];
            lo.resize(P->n_units + 1);
            lo[0] = 0;
            for (int k = 0; k < P->n_units; ++k) {
                const UnitDev& U = P->units[ord[k]];
                lo[k + 1] = lo[k] + ((int64_t)1 << (U.lsum - U.lv[ax]));
            }
            int k0 = 0;
            while (k0 < P->n_units) {
                const int lm = P->units[ord[k0]].lv[ax];
                int k1 = k0;
                while (k1 < P->n_units && P->units[ord[k1]].lv[ax] == lm) ++k1;
                int k = k0;
                for (int64_t s = lo[k0]; s < lo[k1]; s += LINE_BLOCK) {
                    while (s >= lo[k + 1]) ++k;
                    SweepBlk B{};
                    B.line_start = s;
                    B.line_end = std::min<int64_t>(s + LINE_BLOCK, lo[k1]);
                    B.k_start = k;
                    B.lm = lm;
                    P->ax_blk[ax].push_back(B);
                }
                k0 = k1;
            }
        }

        // workspace layout
        size_t o = 0;
        const size_t vb = align_up((size_t)P->total * P->elem, 256);
        for (int v = 0; v < N_VEC; ++v) {
            P->off_vec[v] = o;
            o += vb;
        }
        auto take = [&](size_t bytes) {
            const size_t at = o;
            o = align_up(o + bytes, 256);
            return at;
        };
        P->off_units = take(P->units.size() * sizeof(UnitDev));
        P->off_probs = take(P->probdev.size() * sizeof(ProbDev));
        P->off_tab = take(P->tabd.size() * P->elem);
        P->off_blk = take(P->blk_unit.size() * sizeof(int32_t));
        for (int ax = 0; ax < d; ++ax) {
            P->off_axu[ax] = take(P->ax_units[ax].size() * sizeof(int32_t));
            P->off_axl[ax] = take(P->ax_line_off[ax].size() * sizeof(int64_t));
            P->off_axb[ax] = take(P->ax_blk[ax].size() * sizeof(SweepBlk));
        }
        P->off_coef = take(P->coef.size() * sizeof(double));
        P->off_vals = take((size_t)P->n_units * sizeof(double));
        P->off_valsc = take((size_t)P->n_units * sizeof(double));
        P->ws_bytes = o;
    } catch (const std::bad_alloc&) {
        delete P;
        return fail(AMF_E_NOMEM, "out of host memory while building the plan");
    }
    *out = P;
    return AMF_OK;
}

amf_status amf_plan_info_get(const amf_plan* P, amf_plan_info* out)
{
    if (!P || !out) return fail(AMF_E_INVALID, "null argument");
    out->n_problems = P->n_probs;
    out->n_units = P->n_units;
    out->inner_points = P->total;
    out->stage_updates_per_solve = P->total * (int64_t)P->sch.stages * P->steps * (P->richardson ? 3 : 1);
    out->workspace_bytes = P->ws_bytes;
    out->state_offset = P->off_vec[V_Y];
    out->vector_bytes = (uint64_t)P->total * P->elem;
    out->d = P->d;
    out->precision = P->prec;
    out->n_steps = P->steps;
    out->richardson = P->richardson;
    return AMF_OK;
}

amf_status amf_unit_info(const amf_plan* P, int64_t unit, int32_t* problem, int32_t* levels,
                         double* coef, int64_t* offset)
{
    if (!P) return fail(AMF_E_INVALID, "null plan");
    if (unit < 0 || unit >= P->n_units) return fail(AMF_E_INVALID, "unit out of range");
    const UnitDev& U = P->units[unit];
    if (problem) *problem = U.prob;
    if (levels)
        for (int i = 0; i < P->d; ++i) levels[i] = U.lv[i];
    if (coef) *coef = P->coef[unit];
    if (offset) *offset = U.off;
    return AMF_OK;
}

amf_status amf_plan_bind(amf_plan* P, void* d_ws, uint64_t bytes, void* stream)
{
    if (!P) return fail(AMF_E_INVALID, "null plan");
    if (!d_ws) return fail(AMF_E_INVALID, "null workspace");
    if (bytes < P->ws_bytes) return fail(AMF_E_INVALID, "workspace too small: need " + std::to_string(P->ws_bytes) + " bytes");
    if (((uintptr_t)d_ws & 255u) != 0) return fail(AMF_E_INVALID, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    P->ws = (char*)d_ws;
    P->bound = false;
    P->initialised = false;
    P->have_coarse = false;
    amf_status st;
    if ((st = upload(P->ws + P->off_units, P->units.data(), P->units.size() * sizeof(UnitDev), s))) return st;
    if ((st = upload(P->ws + P->off_probs, P->probdev.data(), P->probdev.size() * sizeof(ProbDev), s))) return st;
    std::vector<float> tf;
    if (P->prec == AMF_FP64) {
        if ((st = upload(P->ws + P->off_tab, P->tabd.data(), P->tabd.size() * 8, s))) return st;
    } else {
        tf = cast_vec<float>(P->tabd);
        if ((st = upload(P->ws + P->off_tab, tf.data(), tf.size() * 4, s))) return st;
    }
    if ((st = upload(P->ws + P->off_blk, P->blk_unit.data(), P->blk_unit.size() * 4, s))) return st;
    for (int ax = 0; ax < P->d; ++ax) {
        if ((st = upload(P->ws + P->off_axu[ax], P->ax_units[ax].data(), P->ax_units[ax].size() * 4, s))) return st;
        if ((st = upload(P->ws + P->off_axl[ax], P->ax_line_off[ax].data(), P->ax_line_off[ax].size() * 8, s))) return st;
        if ((st = upload(P->ws + P->off_axb[ax], P->ax_blk[ax].data(), P->ax_blk[ax].size() * sizeof(SweepBlk), s))) return st;
    }
    if ((st = upload(P->ws + P->off_coef, P->coef.data(), P->coef.size() * 8, s))) return st;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");

    DevPlan& D = P->dev;
    D = DevPlan{};
    D.d = P->d;
    D.n_units = P->n_units;
    D.n_probs = P->n_probs;
    D.total = P->total;
    D.units = (const UnitDev*)(P->ws + P->off_units);
    D.probs = (const ProbDev*)(P->ws + P->off_probs);
    D.tab = P->ws + P->off_tab;
    D.blk_unit = (const int32_t*)(P->ws + P->off_blk);
    D.n_node_blocks = (int64_t)P->blk_unit.size();
    for (int ax = 0; ax < P->d; ++ax) {
        D.ax_units[ax] = (const int32_t*)(P->ws + P->off_axu[ax]);
        D.ax_line_off[ax] = (const int64_t*)(P->ws + P->off_axl[ax]);
        D.ax_blk[ax] = (const SweepBlk*)(P->ws + P->off_axb[ax]);
        D.ax_nblk[ax] = (int64_t)P->ax_blk[ax].size();
    }
    P->bound = true;
    return AMF_OK;
}

}  // extern "C"

namespace {

amf_status check_bound(const amf_plan* P)
{
    if (!P) return fail(AMF_E_INVALID, "null plan");
    if (!P->bound) return fail(AMF_E_STATE, "plan has no bound workspace");
    return AMF_OK;
}

hipEvent_t pool_event(amf_plan* P)
{
    if (P->pool_next == P->pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        P->pool.push_back(e);
    }
    return P->pool[P->pool_next++];
}

// Launch through `fn`, bracketed by events when profiling is on.
template <class Fn>
hipError_t timed(amf_plan* P, int kclass, double bytes, hipStream_t s, Fn&& fn)
{
    if (!P->prof) return fn();
    hipEvent_t a = pool_event(P), b = pool_event(P);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    if ((e = fn()) != hipSuccess) return e;
    if ((e = hipEventRecord(b, s)) != hipSuccess) return e;
    P->recs.push_back({kclass, a, b, bytes});
    return hipSuccess;
}

hipError_t run_stencil(amf_plan* P, int op, const StencilArgs& a, hipStream_t s)
{
    const double nv = (op == OP_F_PAYOFF || op == OP_F_ZERO) ? 2.0 : 3.0;
    return timed(P, AMF_K_STENCIL, nv * P->vbytes(), s,
                 [&] { return launch_stencil(P->dev, P->prec, op, a, s); });
}

hipError_t run_sweep(amf_plan* P, int axis, int epi, const SweepArgs& a, hipStream_t s)
{
    const bool up = epi == EPI_UPDATE;
    return timed(P, up ? AMF_K_SWEEP_UPDATE : AMF_K_SWEEP, (up ? 4.0 : 2.0) * P->vbytes(), s,
                 [&] { return launch_sweep(P->dev, P->prec, axis, epi, a, s); });
}

hipError_t run_init(amf_plan* P, hipStream_t s)
{
    return timed(P, AMF_K_INIT, P->vbytes(), s, [&] { return launch_init(P->dev, P->prec, P->vec(V_Y), s); });
}

hipError_t run_unit_values(amf_plan* P, double* vals, hipStream_t s)
{
    const double b = (double)P->n_units * (double)(1 << P->d) * (double)P->elem + 8.0 * P->n_units;
    return timed(P, AMF_K_UNIT_VALUES, b, s,
                 [&] { return launch_unit_values(P->dev, P->prec, P->vec(V_Y), vals, s); });
}

// One AMFR-W step (eq amfrw) of the 2-stage scheme on every unit.  run selects dt (0: coarse,
// 1: fine half step of the Richardson pair).
amf_status one_step(amf_plan* P, int run, hipStream_t s)
{
    const int d = P->d;
    const int sel_dt = CST_RUN + 3 * run, sel_nu = sel_dt + 1, sel_th = sel_dt + 2;
    void *Y = P->vec(V_Y), *K1 = P->vec(V_K1), *A = P->vec(V_A), *B = P->vec(V_B), *Cb = P->vec(V_C);
    const double a21 = P->sch.a[1 * AMF_MAX_STAGES + 0], q21 = P->sch.q[1 * AMF_MAX_STAGES + 0];
    hipError_t e;
    auto chain = [&](const void* in, void* dst, bool last_update) -> hipError_t {
        // (I - nu dt A_1)..(I - nu dt A_d) applied in axis order; first sweep out of place
        for (int ax = 0; ax < d; ++ax) {
            SweepArgs a{};
            a.in = ax == 0 ? in : dst;
            a.out = dst;
            a.cbuf = Cb;
            a.nudt_sel = sel_nu;
            int epi = EPI_STORE;
            if (last_update && ax == d - 1) {
                epi = EPI_UPDATE;
                a.out = Y;
                a.K1 = K1;
                a.b1 = P->sch.b[0];
                a.b2 = P->sch.b[1];
            }
            hipError_t err = run_sweep(P, ax, epi, a, s);
            if (err != hipSuccess) return err;
        }
        return hipSuccess;
    };
    // ---- stage 1: K^(0) = dt F(Y)
    StencilArgs st{};
    st.X0 = Y;
    st.W = A;
    st.scale_sel = sel_dt;
    if ((e = run_stencil(P, OP_F_PAYOFF, st, s)) != hipSuccess) return hip_fail(e, "stencil");
    if ((e = chain(A, B, false)) != hipSuccess) return hip_fail(e, "sweep");
    // Khat^(0) = 2 K^(0) - K^(d) + theta dt F(K^(d))
    st = StencilArgs{};
    st.X0 = B;
    st.W = A;
    st.scale_sel = sel_th;
    if ((e = run_stencil(P, OP_REFINE, st, s)) != hipSuccess) return hip_fail(e, "stencil");
    if ((e = chain(A, K1, false)) != hipSuccess) return hip_fail(e, "sweep");
    // ---- stage 2: K^(0) = dt F(Y + a21 K1) + q21 K1
    st = StencilArgs{};
    st.X0 = Y;
    st.X1 = K1;
    st.W = A;
    st.a = a21;
    st.q = q21;
    st.scale_sel = sel_dt;
    if ((e = run_stencil(P, OP_STAGE, st, s)) != hipSuccess) return hip_fail(e, "stencil");
    if ((e = chain(A, B, false)) != hipSuccess) return hip_fail(e, "sweep");
    st = StencilArgs{};
    st.X0 = B;
    st.W = A;
    st.scale_sel = sel_th;
    if ((e = run_stencil(P, OP_REFINE, st, s)) != hipSuccess) return hip_fail(e, "stencil");
    // second chain of stage 2 ends in Y += b1 K1 + b2 K2
    if (d == 1) return fail(AMF_E_UNSUPPORTED, "d = 1");
    if ((e = chain(A, B, true)) != hipSuccess) return hip_fail(e, "sweep");
    return AMF_OK;
}

}  // namespace

extern "C" {

amf_status amf_init(amf_plan* P, void* stream)
{
    amf_status st = check_bound(P);
    if (st) return st;
    hipError_t e = run_init(P, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "init");
    P->initialised = true;
    P->have_coarse = false;
    return AMF_OK;
}

amf_status amf_time_step(amf_plan* P, int32_t n, void* stream)
{
    amf_status st = check_bound(P);
    if (st) return st;
    if (!P->initialised) return fail(AMF_E_STATE, "amf_init has not been called");
    if (n < 0) return fail(AMF_E_INVALID, "n must be >= 0");
    for (int i = 0; i < n; ++i)
        if ((st = one_step(P, 0, (hipStream_t)stream))) return st;
    return AMF_OK;
}

amf_status amf_solve(amf_plan* P, void* stream)
{
    amf_status st = check_bound(P);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = amf_init(P, stream))) return st;
    for (int i = 0; i < P->steps; ++i)
        if ((st = one_step(P, 0, s))) return st;
    if (P->richardson) {
        hipError_t e = run_unit_values(P, (double*)(P->ws + P->off_valsc), s);
        if (e != hipSuccess) return hip_fail(e, "unit values");
        if ((e = run_init(P, s)) != hipSuccess) return hip_fail(e, "init");
        for (int i = 0; i < 2 * P->steps; ++i)
            if ((st = one_step(P, 1, s))) return st;
        P->have_coarse = true;
    }
    return AMF_OK;
}

amf_status amf_unit_values(amf_plan* P, double* d_values, void* stream)
{
    amf_status st = check_bound(P);
    if (st) return st;
    if (!d_values) return fail(AMF_E_INVALID, "null output");
    hipError_t e = run_unit_values(P, d_values, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "unit values");
    return AMF_OK;
}

amf_status amf_combine(amf_plan* P, double* d_prices, void* stream)
{
    amf_status st = check_bound(P);
    if (st) return st;
    if (!d_prices) return fail(AMF_E_INVALID, "null output");
    hipStream_t s = (hipStream_t)stream;
    double* vals = (double*)(P->ws + P->off_vals);
    hipError_t e = run_unit_values(P, vals, s);
    if (e != hipSuccess) return hip_fail(e, "unit values");
    const double* coarse = (P->richardson && P->have_coarse) ? (const double*)(P->ws + P->off_valsc) : nullptr;
    e = timed(P, AMF_K_COMBINE, 16.0 * P->n_units, s, [&] {
        return launch_combine(P->dev, (const double*)(P->ws + P->off_coef), vals, coarse, d_prices, s);
    });
    if (e != hipSuccess) return hip_fail(e, "combine");
    return AMF_OK;
}

amf_status amf_state_ptr(const amf_plan* P, void** d_state)
{
    amf_status st = check_bound(P);
    if (st) return st;
    if (!d_state) return fail(AMF_E_INVALID, "null output");
    *d_state = P->vec(V_Y);
    return AMF_OK;
}

amf_status amf_apply_operator(amf_plan* P, const void* d_in, void* d_out, int32_t increment,
                              double scale, void* stream)
{
    amf_status st = check_bound(P);
    if (st) return st;
    if (!d_in || !d_out || d_in == d_out) return fail(AMF_E_INVALID, "need distinct input and output vectors");
    StencilArgs a{};
    a.X0 = d_in;
    a.W = d_out;
    a.scale = scale;
    a.scale_sel = -1;
    hipError_t e = launch_stencil(P->dev, P->prec, increment ? OP_F_ZERO : OP_F_PAYOFF, a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "stencil");
    return AMF_OK;
}

amf_status amf_axis_solve(amf_plan* P, int32_t axis, const void* d_in, void* d_out, void* stream)
{
    amf_status st = check_bound(P);
    if (st) return st;
    if (axis < 0 || axis >= P->d) return fail(AMF_E_INVALID, "axis out of range");
    if (!d_in || !d_out) return fail(AMF_E_INVALID, "null vector");
    SweepArgs a{};
    a.in = d_in;
    a.out = d_out;
    a.cbuf = P->vec(V_C);
    a.nudt_sel = CST_RUN + 1;
    hipError_t e = launch_sweep(P->dev, P->prec, axis, EPI_STORE, a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "sweep");
    return AMF_OK;
}

amf_status amf_profile_begin(amf_plan* P)
{
    if (!P) return fail(AMF_E_INVALID, "null plan");
    P->prof = true;
    P->recs.clear();
    P->pool_next = 0;
    return AMF_OK;
}

amf_status amf_profile_end(amf_plan* P, amf_kernel_stat* stats)
{
    if (!P || !stats) return fail(AMF_E_INVALID, "null argument");
    for (int k = 0; k < AMF_K_COUNT; ++k) {
        stats[k] = amf_kernel_stat{};
        stats[k].kernel = k;
    }
    P->prof = false;
    if (!P->recs.empty()) {
        hipError_t e = hipEventSynchronize(P->recs.back().b);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    }
    for (const auto& r : P->recs) {
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        stats[r.kclass].launches += 1;
        stats[r.kclass].total_ms += ms;
        stats[r.kclass].algo_bytes += r.bytes;
    }
    P->recs.clear();
    P->pool_next = 0;
    return AMF_OK;
}

void amf_plan_destroy(amf_plan* P) { delete P; }

}  // extern "C"
