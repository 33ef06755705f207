// Host side of libamfrw: descriptor validation, enumeration of the combination technique's
// component grids, 1-D coefficient tables, workspace layout and the C ABI of include/amfrw.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
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

// Grid vectors: the solution W = Y - g, two work vectors, F(g), then the stages K_1 .. K_{s-1} of
// the scheme, and for s > 2 two combination vectors (sum_j a_rj K_j, sum_j q_rj K_j).
enum VecId { V_W = 0, V_A = 1, V_B = 2, V_G = 3, V_K0 = 4 };
constexpr int MAX_VEC = V_K0 + AMF_MAX_STAGES - 1 + 2;

struct amf_plan {
    int d = 0, prec = 0, steps = 0, richardson = 0, n_probs = 0, n_units = 0;
    amf_scheme sch{};
    amf_grid_spec grid{};
    int n_vec = 0;                         // grid vectors in the workspace
    int v_z = -1, v_q = -1;                // combination vectors (s > 2)
    std::vector<amf_problem> probs;
    std::vector<UnitDev> units;            // n_units + sentinel
    std::vector<double> coef;              // combination coefficient per unit
    std::vector<double> tabd;              // coefficient tables in FP64
    std::vector<double> facd;              // Thomas factor tables in FP64 (run 0, then run 1)
    int64_t fac_run = 0;                   // elements per run in facd
    std::vector<ProbDev> probdev;
    std::vector<int32_t> blk_unit;
    std::vector<int32_t> blk_unit_r[4];    // node blocks of NODE_BLOCK * {1, 2, 4, 8} nodes
    std::vector<VecBlk> vblk;              // operator blocks by axis-1 line class (VB_LISTS lists)
    int64_t vblk_off[VB_LISTS]{}, vblk_n[VB_LISTS]{};
    size_t off_vblk = 0;
    int stencil_r = 1, min_m0 = 1, max_m0 = 1, xcd = 1;
    int fuse0 = 0;                         // fused axis-0 solve in the operator launches
    bool res_ok = false;                   // every unit fits the unit-resident schedule
    int resident = 0, res_lds_len = 0, res_tab_len = 0;
    std::vector<int32_t> ax_units[MAXD];
    std::vector<int64_t> ax_line_off[MAXD];
    std::vector<SweepBlk> ax_blk[MAXD];
    double ax_short_frac[MAXD]{};          // share of inner points on lines up to 2^SHORT_LM
    int ax_vec[MAXD]{};                    // lines per thread of the short strided sweep (1 or 16 B / elem)
    int64_t total = 0;                     // elements per grid vector (with alignment padding)
    int64_t inner = 0;                     // inner points over all units

    // marching operator (d <= 4): blocks and the largest plane slot
    std::vector<MarchBlk> march_blk, march_blk_x;
    int march_lp = 0, march = 0;
    size_t off_march = 0, off_march_x = 0;
    // W = P solves: hyperplanes of axis-0 lines per unit (built only for w_matrix = AMF_W_LOWER)
    std::vector<int32_t> gs_unit_plane0, gs_lines;
    std::vector<int64_t> gs_plane_line0;
    size_t off_gsu = 0, off_gsp = 0, off_gsl = 0;

    size_t off_vec[MAX_VEC]{}, off_units = 0, off_probs = 0, off_tab = 0, off_fac = 0, off_blk = 0;
    size_t off_blkr[4]{};
    size_t off_axu[MAXD]{}, off_axl[MAXD]{}, off_axb[MAXD]{};
    size_t off_coef = 0, off_vals = 0, off_valsc = 0, off_flag = 0;
    size_t core_bytes = 0;                 // everything but the fallback staging area
    size_t off_fb = 0, ws_bytes = 0;       // staging of routed prices and their indices
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

    // whole-solve hipGraph (captured on first use, replayed by amf_solve)
    bool graph_on = false, graph_valid = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t cap_stream = nullptr;

    void* vec(int v) const { return ws + off_vec[v]; }
    double vbytes() const { return (double)total * (double)elem; }

    void drop_graph()
    {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
        graph_valid = false;
    }

    ~amf_plan()
    {
        drop_graph();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
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
    if (p.boundary != AMF_BC_NEUMANN && p.boundary != AMF_BC_DIRICHLET)
        return fail(AMF_E_INVALID, "unknown boundary kind" + at);
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

// Thomas factors of (I - nu dt A_axis) along one line (Lemma lema:ls) from the FP64 diagonal
// weights delta_r = d_axis/h^2: appends inv_r = 1/pivot_r, a_r inv_r, c'_r (three blocks of M).
// dir: the last node is a Dirichlet face (eq bound1_0), whose row is the identity.
void append_factors(std::vector<double>& f, const std::vector<double>& delta, double nudt, bool dir)
{
    const int M = (int)delta.size();
    const size_t b = f.size();
    f.resize(b + 3 * (size_t)M);
    double cprev = 0.0;
    for (int r = 0; r < M; ++r) {
        const double nd = (dir && r == M - 1) ? 0.0 : nudt * delta[r];
        const double bb = 1.0 + 2.0 * nd;
        const double a = (r == 0) ? 0.0 : ((r == M - 1) ? -2.0 * nd : -nd);
        const double c = (r == M - 1) ? 0.0 : -nd;
        const double inv = 1.0 / (bb - a * cprev);
        const double cp = c * inv;
        f[b + r] = inv;
        f[b + M + r] = a * inv;
        f[b + 2 * M + r] = cp;
        cprev = cp;
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
    out->w_matrix = AMF_W_AMF;
    return AMF_OK;
}

amf_status amf_scheme_theta_gs(double theta, int32_t stages, amf_scheme* out)
{
    if (!out) return fail(AMF_E_INVALID, "null scheme");
    if (!(theta > 0.0 && theta <= 1.0)) return fail(AMF_E_INVALID, "theta must lie in (0, 1]");
    if (stages < 1 || stages > AMF_MAX_STAGES) return fail(AMF_E_INVALID, "stages must lie in [1, 6]");
    std::memset(out, 0, sizeof(*out));
    out->struct_size = sizeof(amf_scheme);
    out->stages = stages;
    for (int r = 0; r < stages; ++r) {
        out->b[r] = 1.0;
        for (int j = 0; j < r; ++j) {
            out->a[r * AMF_MAX_STAGES + j] = theta;
            out->q[r * AMF_MAX_STAGES + j] = -1.0;
        }
    }
    out->theta = theta;
    out->nu = theta;
    out->w_matrix = AMF_W_LOWER;
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
    if (scheme->stages < 1 || scheme->stages > AMF_MAX_STAGES) return fail(AMF_E_INVALID, "stages must lie in [1, 6]");
    if (scheme->w_matrix != AMF_W_AMF && scheme->w_matrix != AMF_W_LOWER) return fail(AMF_E_INVALID, "unknown w_matrix");
    if (!(scheme->theta > 0.0) || !std::isfinite(scheme->theta)) return fail(AMF_E_INVALID, "theta must be > 0");
    if (scheme->w_matrix == AMF_W_AMF && (!(scheme->nu > 0.0) || !std::isfinite(scheme->nu)))
        return fail(AMF_E_INVALID, "nu must be > 0");
    for (int r = 0; r < scheme->stages; ++r) {
        if (!std::isfinite(scheme->b[r])) return fail(AMF_E_INVALID, "scheme coefficients must be finite");
        for (int j = 0; j < r; ++j)
            if (!std::isfinite(scheme->a[r * AMF_MAX_STAGES + j]) || !std::isfinite(scheme->q[r * AMF_MAX_STAGES + j]))
                return fail(AMF_E_INVALID, "scheme coefficients must be finite");
    }
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
            if (grid->levels[i] < 0 || grid->levels[i] > MAX_LEVEL)
                return fail(AMF_E_INVALID, "levels must lie in [0, " + std::to_string(MAX_LEVEL) + "]");
            row[i] = grid->levels[i];
            s += row[i];
        }
        if (s > 30) return fail(AMF_E_INVALID, "full grid too large (sum of levels > 30)");
        glv.push_back(row);
        gcf.push_back(1.0);
    } else {
        if (grid->psi < 0 || grid->psi > 8) return fail(AMF_E_INVALID, "psi must lie in [0, 8]");
        if (grid->n < d - 1) return fail(AMF_E_INVALID, "n must be >= d-1 (combination coefficients sum to 1)");
        if (grid->psi + grid->n > MAX_LEVEL || d * grid->psi + grid->n > 30)
            return fail(AMF_E_INVALID, "combination level too large");
        enumerate_grids(d, grid->n, grid->psi, glv, gcf);
    }
    if (scheme->w_matrix == AMF_W_LOWER)
        for (const std::vector<int>& row : glv)
            if (row[0] > CONTIG_PART_LM)
                return fail(AMF_E_UNSUPPORTED, "the W = P solve takes axis-1 levels up to " + std::to_string(CONTIG_PART_LM));

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
        P->grid = *grid;
        P->probs.assign(probs, probs + n_probs);
        {
            const int S = scheme->stages;
            P->n_vec = V_K0 + (S - 1);
            if (S > 2) {
                P->v_z = P->n_vec++;
                P->v_q = P->n_vec++;
            }
        }
        const int ng = (int)glv.size();
        const int64_t nu64 = (int64_t)ng * n_probs;
        if (nu64 > (int64_t)1 << 30) {
            delete P;
            return fail(AMF_E_INVALID, "too many units");
        }
        P->n_units = (int)nu64;

        // Per problem (independent, built on host threads): a constant block and (axis, level)
        // coefficient blocks, the Thomas factor tables of both runs, and each grid's table
        // indices, all relative to the problem's own buffers; then concatenated in problem order.
        struct ProbTables {
            ProbDev pd{};
            std::vector<double> tab;
            std::vector<double> fac[2];
            std::vector<int64_t> unit_tab, unit_fac;   // [g * d + i], relative
        };
        std::vector<ProbTables> pt((size_t)n_probs);
        auto build_problem = [&](int p) {
            const amf_problem& pr = probs[p];
            ProbTables& T = pt[(size_t)p];
            ProbDev& pd = T.pd;
            for (int i = 0; i < d; ++i) {
                pd.xmax[i] = pr.x_max[i];
                pd.xeval[i] = pr.x_eval[i];
            }
            for (int i = 0; i < d - 1; ++i) pd.tau[i] = pr.tau[i];
            pd.K = pr.strike;
            pd.discount = pr.discount;
            pd.payoff = pr.payoff;
            pd.dirichlet = pr.boundary == AMF_BC_DIRICHLET ? 1 : 0;
            pd.cst = 0;
            pd.unit_begin = p * ng;
            pd.unit_end = (p + 1) * ng;
            std::vector<double>& tab = T.tab;
            tab.assign(CST_SIZE, 0.0);
            for (int i = 0; i < d - 1; ++i) {
                for (int k = 0; k < d - 1; ++k) tab[CST_RHO + i * MAXD + k] = pr.rho[i * RHO_LD + k];
                tab[CST_SPHI + i] = pr.sigma * pr.phi[i];
            }
            const double dt = pr.maturity / (double)n_steps;
            for (int run = 0; run < 2; ++run) {
                const double h = run == 0 ? dt : 0.5 * dt;
                tab[CST_RUN + 3 * run + 0] = h;
                tab[CST_RUN + 3 * run + 1] = scheme->nu * h;
                tab[CST_RUN + 3 * run + 2] = scheme->theta * h;
            }
            // axis tables for every level in use on that axis
            std::vector<int64_t> blk_of[MAXD];
            for (int i = 0; i < d; ++i) blk_of[i].assign(MAX_LEVEL + 1, -1);
            T.unit_tab.assign((size_t)ng * d, 0);
            for (int g = 0; g < ng; ++g)
                for (int i = 0; i < d; ++i) {
                    const int L = glv[g][i];
                    if (blk_of[i][L] < 0) {
                        blk_of[i][L] = (int64_t)tab.size();
                        append_axis_table(tab, pr, i, L);
                    }
                    T.unit_tab[(size_t)g * d + i] = blk_of[i][L];
                }
            // Thomas factors per (axis, level, V level) in use, both runs (axis 0: the fused solve)
            constexpr int NL = MAX_LEVEL + 1;
            std::vector<std::vector<int64_t>> fac_of(d, std::vector<int64_t>(NL * NL, -1));
            // FP64 weights delta_r = d_ax / h_ax^2 along a line (as the coefficient tables hold them)
            std::vector<double> dl;
            auto delta_of = [&](int ax, int L, int LV, int jv, const std::vector<double>& t,
                                const std::vector<double>& tv) -> const std::vector<double>& {
                const int M = 1 << L, MV = 1 << LV;
                dl.resize(M);
                for (int r = 0; r < M; ++r)
                    dl[r] = (ax < d - 1) ? t[r] * tv[jv] : tv[MV] * tv[r];
                return dl;
            };
            T.unit_fac.assign((size_t)ng * d, 0);
            std::vector<double> t, tv;
            for (int g = 0; g < ng; ++g)
                for (int i = 0; i < d; ++i) {
                    const int L = glv[g][i], LV = glv[g][d - 1];
                    const int key = (i < d - 1) ? L * NL + LV : L * NL + L;
                    if (fac_of[i][key] < 0) {
                        fac_of[i][key] = (int64_t)T.fac[0].size();
                        const int nlines = (i < d - 1) ? (1 << LV) : 1;
                        t.clear();
                        tv.clear();
                        append_axis_table(t, pr, i, L);
                        append_axis_table(tv, pr, d - 1, LV);
                        for (int run = 0; run < 2; ++run) {
                            const double h = run == 0 ? pr.maturity / (double)n_steps : 0.5 * pr.maturity / (double)n_steps;
                            for (int jv = 0; jv < nlines; ++jv)
                                append_factors(T.fac[run], delta_of(i, L, LV, jv, t, tv), scheme->nu * h,
                                               pr.boundary == AMF_BC_DIRICHLET && i < d - 1);
                        }
                    }
                    T.unit_fac[(size_t)g * d + i] = fac_of[i][key];
                }
        };
        {
            // problems on up to 16 host threads; any exception is rethrown here
            const int nt = std::max(1, std::min<int>({n_probs, 16, (int)std::max(1u, std::thread::hardware_concurrency())}));
            std::vector<std::exception_ptr> errs((size_t)nt);
            std::vector<std::thread> pool;
            for (int w = 0; w < nt; ++w)
                pool.emplace_back([&, w] {
                    try {
                        for (int p = w; p < n_probs; p += nt) build_problem(p);
                    } catch (...) {
                        errs[(size_t)w] = std::current_exception();
                    }
                });
            for (std::thread& th : pool) th.join();
            for (std::exception_ptr& e : errs)
                if (e) std::rethrow_exception(e);
        }
        // concatenate in problem order (buffers sized once); units in problem order, grid order
        // within a problem; the run-1 factor tables follow all run-0 tables
        int64_t ntab = 0, nfac = 0;
        for (const ProbTables& T : pt) {
            ntab += (int64_t)T.tab.size();
            nfac += (int64_t)T.fac[0].size();
        }
        if (ntab > (int64_t)INT32_MAX / 2 || nfac > (int64_t)INT32_MAX) throw std::bad_alloc();
        P->tabd.resize((size_t)ntab);
        P->facd.resize((size_t)(2 * nfac));
        P->fac_run = nfac;
        P->units.reserve((size_t)P->n_units + 1);
        P->coef.reserve((size_t)P->n_units);
        P->probdev.reserve((size_t)n_probs);
        int64_t tab0 = 0, fac0 = 0;
        for (int p = 0; p < n_probs; ++p) {
            ProbTables& T = pt[(size_t)p];
            T.pd.cst = (int32_t)tab0;
            std::copy(T.tab.begin(), T.tab.end(), P->tabd.begin() + tab0);
            std::copy(T.fac[0].begin(), T.fac[0].end(), P->facd.begin() + fac0);
            std::copy(T.fac[1].begin(), T.fac[1].end(), P->facd.begin() + nfac + fac0);
            P->probdev.push_back(T.pd);
            for (int g = 0; g < ng; ++g) {
                UnitDev U{};
                // offsets are multiples of min(M_0, 1024) as well, so that node blocks of the
                // fused operator (NODE_BLOCK * R >= M_0 nodes) never split an axis-0 line
                const int64_t al = std::max<int64_t>(UNIT_ALIGN, std::min<int64_t>(1024, (int64_t)1 << glv[g][0]));
                P->total = (P->total + al - 1) / al * al;
                U.off = P->total;
                U.prob = p;
                int ls = 0;
                for (int i = 0; i < d; ++i) {
                    U.lv[i] = (int8_t)glv[g][i];
                    U.tab[i] = (int32_t)(tab0 + T.unit_tab[(size_t)g * d + i]);
                    const int64_t f = fac0 + T.unit_fac[(size_t)g * d + i];
                    if (f > INT32_MAX) throw std::bad_alloc();
                    U.fac[i] = (int32_t)f;
                    ls += glv[g][i];
                }
                U.lsum = ls;
                P->units.push_back(U);
                P->coef.push_back(gcf[g]);
                P->total += (int64_t)1 << ls;
                P->inner += (int64_t)1 << ls;
            }
            tab0 += (int64_t)T.tab.size();
            fac0 += (int64_t)T.fac[0].size();
            std::vector<double>().swap(T.tab);
            std::vector<double>().swap(T.fac[0]);
            std::vector<double>().swap(T.fac[1]);
        }
        P->total = (P->total + UNIT_ALIGN - 1) / UNIT_ALIGN * UNIT_ALIGN;
        UnitDev sentinel{};
        sentinel.off = P->total;
        P->units.push_back(sentinel);

        // node blocks -> first unit
        auto block_table = [&](int64_t per, std::vector<int32_t>& tbl) {
            const int64_t nb = (P->total + per - 1) / per;
            tbl.resize(nb);
            int u = 0;
            for (int64_t b = 0; b < nb; ++b) {
                const int64_t g0 = b * per;
                while (g0 >= P->units[u + 1].off) ++u;
                tbl[b] = u;
            }
        };
        block_table(NODE_BLOCK, P->blk_unit);
        for (int k = 0; k < 4; ++k) block_table((int64_t)NODE_BLOCK << k, P->blk_unit_r[k]);
        // operator blocks of R nodes per thread over the runs of consecutive units of one axis-1
        // line class; unit offsets are multiples of min(M_1, 1024) >= R, so every thread's R
        // nodes lie on one line
        auto vb_list = [&](int id, int R, auto pred) {
            P->vblk_off[id] = (int64_t)P->vblk.size();
            const int64_t per = (int64_t)NODE_BLOCK * R;
            for (int u = 0; u < P->n_units;) {
                if (!pred(u)) {
                    ++u;
                    continue;
                }
                int v = u;
                while (v < P->n_units && pred(v)) ++v;
                const int64_t g1 = P->units[v - 1].off + ((int64_t)1 << P->units[v - 1].lsum);
                int w = u;
                for (int64_t g = P->units[u].off; g < g1; g += per) {
                    while (P->units[w + 1].off <= g) ++w;
                    P->vblk.push_back(VecBlk{g, g1, (int32_t)w, 0});
                }
                u = v;
            }
            P->vblk_n[id] = (int64_t)P->vblk.size() - P->vblk_off[id];
        };
        for (int R = 1; R <= 4; R *= 2) vb_list(vb_exact(R), R, [&](int u) { return P->units[u].lv[0] == (R == 1 ? 0 : R == 2 ? 1 : 2); });
        for (int R = 1; R <= 8; R *= 2) vb_list(vb_atleast(R), R, [&](int u) { return (1 << P->units[u].lv[0]) >= R; });
        if ((int64_t)P->vblk.size() > (int64_t)INT32_MAX) throw std::bad_alloc();
        // time-loop operator: R consecutive axis-0 nodes per thread, R <= every unit's M_0
        int min_m0 = 1 << MAX_LEVEL, max_m0 = 1;
        for (int u = 0; u < P->n_units; ++u) {
            min_m0 = std::min(min_m0, 1 << P->units[u].lv[0]);
            max_m0 = std::max(max_m0, 1 << P->units[u].lv[0]);
        }
        P->min_m0 = min_m0;
        P->max_m0 = max_m0;
        int max_lsum = 0;
        for (int u = 0; u < P->n_units; ++u) max_lsum = std::max(max_lsum, (int)P->units[u].lsum);
        P->res_ok = max_lsum <= (precision == AMF_FP64 ? RES_MAX_LSUM_F64 : RES_MAX_LSUM_F32) &&
                    scheme->stages == 2 && scheme->w_matrix == AMF_W_AMF;
        // unit-resident LDS: four vectors of axis-1 rows at pitch res_pitch(M_1), then the unit's
        // 1-D coefficient tables (3 M_i per rate axis, M_V + 2 for V)
        P->res_lds_len = 0;
        P->res_tab_len = 0;
        for (int u = 0; u < P->n_units; ++u) {
            const UnitDev& U = P->units[u];
            const int m0 = 1 << U.lv[0];
            P->res_lds_len = std::max(P->res_lds_len, ((1 << U.lsum) / m0) * res_pitch(m0));
            int tl = 0;
            for (int i = 0; i < d; ++i) tl += i < d - 1 ? 3 * (1 << U.lv[i]) : (1 << U.lv[i]) + 2;
            P->res_tab_len = std::max(P->res_tab_len, tl);
        }
        const int rmax = precision == AMF_FP64 ? STENCIL_R_F64 : STENCIL_R_F32;
        P->stencil_r = rmax;                   // each unit runs at min(stencil_r, M_1)
        // per axis (one host thread each): units ordered by M_axis, line offsets, blocks that
        // never mix line lengths
        auto build_axis = [&](int ax) {
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
            int64_t short_pts = 0;
            for (int u = 0; u < P->n_units; ++u)
                if (P->units[u].lv[ax] <= SHORT_LM) short_pts += (int64_t)1 << P->units[u].lsum;
            P->ax_short_frac[ax] = P->inner > 0 ? (double)short_pts / (double)P->inner : 0.0;
            // strided lines: V = 16 B / elem adjacent lines carried as one vector per row.  Short
            // lines: per block, when each of its units has runs of at least V adjacent lines on
            // this axis (E = 2^(levels below the axis) >= V); long lines: when every unit has.
            const int vw = ax > 0 ? 16 / (int)P->elem : 1;
            auto unit_vec_ok = [&](int u) {
                int S = 0;
                for (int i = 0; i < ax; ++i) S += P->units[u].lv[i];
                return vw > 1 && (1 << S) >= vw;
            };
            int vec = vw;
            for (int u = 0; u < P->n_units && vec > 1; ++u)
                if (!unit_vec_ok(u)) vec = 1;
            P->ax_vec[ax] = vec;
            int k0 = 0;
            while (k0 < P->n_units) {
                const int lm = P->units[ord[k0]].lv[ax];
                int k1 = k0;
                while (k1 < P->n_units && P->units[ord[k1]].lv[ax] == lm) ++k1;
                if (ax > 0 && lm <= SHORT_LM) {
                    // runs of units with the same vector eligibility, blocks of LINE_BLOCK threads
                    int ka = k0;
                    while (ka < k1) {
                        const bool ok = unit_vec_ok(ord[ka]);
                        int kb = ka;
                        while (kb < k1 && unit_vec_ok(ord[kb]) == ok) ++kb;
                        const int v = ok ? vw : 1;
                        const int slots = lm <= PAIR_LM && ax < d - 1 ? 2 : 1;   // the update runs on axis d - 1
                        const int per = LINE_BLOCK * v * slots;
                        int k = ka;
                        for (int64_t s = lo[ka]; s < lo[kb]; s += per) {
                            while (s >= lo[k + 1]) ++k;
                            SweepBlk B{};
                            B.line_start = s;
                            B.line_end = std::min<int64_t>(s + per, lo[kb]);
                            B.k_start = k;
                            B.lm = lm;
                            B.vec = v;
                            B.slots = slots;
                            P->ax_blk[ax].push_back(B);
                        }
                        ka = kb;
                    }
                    k0 = k1;
                    continue;
                }
                int k = k0;
                // axis 0 lines longer than 2^CONTIG_REG_LM take M/SEG lanes each (up to
                // 2^CONTIG_PART_LM); longer strided lines, and axis-0 lines beyond that: M/seg_rows
                // threads per line slot in blocks of SEG_BLOCK threads, or one thread per line
                int per = LINE_BLOCK;
                const int lv_vec = ax > 0 ? vec : 1;
                const int ss = seg_rows((int)P->elem, lv_vec);
                const bool seg_solver = (ax > 0 && lm > SHORT_LM) || (ax == 0 && lm > CONTIG_PART_LM);
                if (ax == 0 && lm > CONTIG_REG_LM && lm <= CONTIG_PART_LM) per = LINE_BLOCK / ((1 << lm) / SEG);
                else if (seg_solver)
                    per = lm <= seg_max_lm((int)P->elem, lv_vec) ? ((SEG_BLOCK * ss) >> lm) * lv_vec : lv_vec;
                for (int64_t s = lo[k0]; s < lo[k1]; s += per) {
                    while (s >= lo[k + 1]) ++k;
                    SweepBlk B{};
                    B.line_start = s;
                    B.line_end = std::min<int64_t>(s + per, lo[k1]);
                    B.k_start = k;
                    B.lm = lm;
                    B.vec = ax > 0 ? vec : 1;
                    P->ax_blk[ax].push_back(B);
                }
                k0 = k1;
            }
        };
        {
            std::vector<std::exception_ptr> errs((size_t)d);
            std::vector<std::thread> pool;
            for (int ax = 0; ax < d; ++ax)
                pool.emplace_back([&, ax] {
                    try {
                        build_axis(ax);
                    } catch (...) {
                        errs[(size_t)ax] = std::current_exception();
                    }
                });
            for (std::thread& th : pool) th.join();
            for (std::exception_ptr& e : errs)
                if (e) std::rethrow_exception(e);
        }

        // W = P: per unit, its axis-0 lines bucketed by the hyperplane h = sum_{i>=1} i (j_i - 1)
        if (scheme->w_matrix == AMF_W_LOWER) {
            P->gs_unit_plane0.assign((size_t)P->n_units + 1, 0);
            P->gs_plane_line0.push_back(0);
            std::vector<int32_t> hp, cnt, at;
            for (int u = 0; u < P->n_units; ++u) {
                const UnitDev& U = P->units[u];
                const int nl = 1 << (U.lsum - U.lv[0]);
                int planes = 1;
                for (int i = 1; i < d; ++i) planes += i * ((1 << U.lv[i]) - 1);
                hp.assign((size_t)nl, 0);
                cnt.assign((size_t)planes, 0);
                for (int l = 0; l < nl; ++l) {
                    int h = 0, sh = 0;
                    for (int i = 1; i < d; ++i) {
                        h += i * ((l >> sh) & ((1 << U.lv[i]) - 1));
                        sh += U.lv[i];
                    }
                    hp[(size_t)l] = h;
                    ++cnt[(size_t)h];
                }
                at.assign((size_t)planes, 0);
                const int64_t base = (int64_t)P->gs_lines.size();
                int64_t run = base;
                for (int h = 0; h < planes; ++h) {
                    at[(size_t)h] = (int32_t)(run - base);
                    run += cnt[(size_t)h];
                    P->gs_plane_line0.push_back(run);
                }
                P->gs_lines.resize((size_t)run);
                for (int l = 0; l < nl; ++l) P->gs_lines[(size_t)(base + at[(size_t)hp[(size_t)l]]++)] = l;
                P->gs_unit_plane0[(size_t)u + 1] = P->gs_unit_plane0[(size_t)u] + planes;
                if ((int64_t)P->gs_unit_plane0[(size_t)u + 1] > INT32_MAX / 2) throw std::bad_alloc();
            }
        }

        // marching operator blocks (d <= 4)
        if (d <= 4) {
            std::vector<int8_t> lvs((size_t)P->n_units * MAXD);
            for (int u = 0; u < P->n_units; ++u)
                for (int i = 0; i < MAXD; ++i) lvs[(size_t)u * MAXD + i] = P->units[u].lv[i];
            march_blocks(d, P->n_units, lvs.data(), MAXD, (int)P->elem, P->march_blk);
            // the operator is offered only when every tile fits its LDS slot and every V plane of
            // a unit is addressable with 32-bit byte offsets (its buffer accesses)
            bool ok = (int64_t)P->march_blk.size() <= (int64_t)INT32_MAX / 2;
            for (const MarchBlk& B : P->march_blk) {
                const int lt[3] = {B.lt[0], B.lt[1], B.lt[2]};
                const int slot = march_slot_elems(d, lt);
                const UnitDev& U = P->units[B.unit];
                int64_t plane = (int64_t)P->elem;
                for (int i = 0; i < d - 1; ++i) plane <<= U.lv[i];
                ok = ok && slot <= MARCH_MAX_PLANE && plane < (int64_t)MARCH_NONE;
                P->march_lp = std::max(P->march_lp, slot);
            }
            if (ok) {
                march_order_xcd(P->march_blk, NXCD, P->march_blk_x);
            } else {
                std::vector<MarchBlk>().swap(P->march_blk);
                P->march_lp = 0;
            }
        }

        // workspace layout
        size_t o = 0;
        const size_t vb = align_up((size_t)P->total * P->elem, 256);
        for (int v = 0; v < P->n_vec; ++v) {
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
        P->off_fac = take(P->facd.size() * P->elem);
        P->off_blk = take(P->blk_unit.size() * sizeof(int32_t));
        for (int k = 0; k < 4; ++k) P->off_blkr[k] = take(P->blk_unit_r[k].size() * sizeof(int32_t));
        P->off_vblk = take(P->vblk.size() * sizeof(VecBlk));
        for (int ax = 0; ax < d; ++ax) {
            P->off_axu[ax] = take(P->ax_units[ax].size() * sizeof(int32_t));
            P->off_axl[ax] = take(P->ax_line_off[ax].size() * sizeof(int64_t));
            P->off_axb[ax] = take(P->ax_blk[ax].size() * sizeof(SweepBlk));
        }
        P->off_march = take(P->march_blk.size() * sizeof(MarchBlk));
        P->off_march_x = take(P->march_blk_x.size() * sizeof(MarchBlk));
        P->off_gsu = take(P->gs_unit_plane0.size() * sizeof(int32_t));
        P->off_gsp = take(P->gs_plane_line0.size() * sizeof(int64_t));
        P->off_gsl = take(P->gs_lines.size() * sizeof(int32_t));
        P->off_coef = take(P->coef.size() * sizeof(double));
        P->off_vals = take((size_t)P->n_units * sizeof(double));
        P->off_valsc = take((size_t)P->n_units * sizeof(double));
        P->off_flag = take(sizeof(int32_t));
        P->core_bytes = o;
        P->off_fb = take((size_t)n_probs * (sizeof(double) + sizeof(int32_t)));
        P->ws_bytes = o;
    } catch (const std::bad_alloc&) {
        delete P;
        return fail(AMF_E_NOMEM, "out of host memory while building the plan");
    } catch (const std::exception& e) {
        delete P;
        return fail(AMF_E_INVALID, std::string("plan construction failed: ") + e.what());
    }
    *out = P;
    return AMF_OK;
}

amf_status amf_plan_info_get(const amf_plan* P, amf_plan_info* out)
{
    if (!P || !out) return fail(AMF_E_INVALID, "null argument");
    out->n_problems = P->n_probs;
    out->n_units = P->n_units;
    out->inner_points = P->inner;
    out->stage_updates_per_solve = P->inner * (int64_t)P->sch.stages * P->steps * (P->richardson ? 3 : 1);
    out->workspace_bytes = P->ws_bytes;
    out->state_offset = P->off_vec[V_W];
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

}  // extern "C"

namespace {

// Upload the plan's tables into device memory at d_ws (at least core_bytes; 256-byte aligned) and
// point the device view there.  Synchronises the stream.
amf_status bind_impl(amf_plan* P, void* d_ws, hipStream_t s)
{
    P->drop_graph();
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
    std::vector<float> ff;
    if (P->prec == AMF_FP64) {
        if ((st = upload(P->ws + P->off_fac, P->facd.data(), P->facd.size() * 8, s))) return st;
    } else {
        ff = cast_vec<float>(P->facd);
        if ((st = upload(P->ws + P->off_fac, ff.data(), ff.size() * 4, s))) return st;
    }
    if ((st = upload(P->ws + P->off_blk, P->blk_unit.data(), P->blk_unit.size() * 4, s))) return st;
    for (int k = 0; k < 4; ++k)
        if ((st = upload(P->ws + P->off_blkr[k], P->blk_unit_r[k].data(), P->blk_unit_r[k].size() * 4, s))) return st;
    if ((st = upload(P->ws + P->off_vblk, P->vblk.data(), P->vblk.size() * sizeof(VecBlk), s))) return st;
    for (int ax = 0; ax < P->d; ++ax) {
        if ((st = upload(P->ws + P->off_axu[ax], P->ax_units[ax].data(), P->ax_units[ax].size() * 4, s))) return st;
        if ((st = upload(P->ws + P->off_axl[ax], P->ax_line_off[ax].data(), P->ax_line_off[ax].size() * 8, s))) return st;
        if ((st = upload(P->ws + P->off_axb[ax], P->ax_blk[ax].data(), P->ax_blk[ax].size() * sizeof(SweepBlk), s))) return st;
    }
    if ((st = upload(P->ws + P->off_march, P->march_blk.data(), P->march_blk.size() * sizeof(MarchBlk), s))) return st;
    if ((st = upload(P->ws + P->off_march_x, P->march_blk_x.data(), P->march_blk_x.size() * sizeof(MarchBlk), s)))
        return st;
    if ((st = upload(P->ws + P->off_gsu, P->gs_unit_plane0.data(), P->gs_unit_plane0.size() * 4, s))) return st;
    if ((st = upload(P->ws + P->off_gsp, P->gs_plane_line0.data(), P->gs_plane_line0.size() * 8, s))) return st;
    if ((st = upload(P->ws + P->off_gsl, P->gs_lines.data(), P->gs_lines.size() * 4, s))) return st;
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
    D.fac = P->ws + P->off_fac;
    D.fac_run_stride = P->fac_run;
    D.blk_unit = (const int32_t*)(P->ws + P->off_blk);
    D.n_node_blocks = (int64_t)P->blk_unit.size();
    D.stencil_r = P->stencil_r;
    D.xcd = P->xcd;
    for (int k = 0; k < 4; ++k) {
        D.blk_unit_r[k] = (const int32_t*)(P->ws + P->off_blkr[k]);
        D.n_blocks_r[k] = (int64_t)P->blk_unit_r[k].size();
    }
    D.vblk = (const VecBlk*)(P->ws + P->off_vblk);
    for (int k = 0; k < VB_LISTS; ++k) {
        D.vblk_off[k] = P->vblk_off[k];
        D.vblk_n[k] = P->vblk_n[k];
    }
    for (int ax = 0; ax < P->d; ++ax) {
        D.ax_units[ax] = (const int32_t*)(P->ws + P->off_axu[ax]);
        D.ax_line_off[ax] = (const int64_t*)(P->ws + P->off_axl[ax]);
        D.ax_blk[ax] = (const SweepBlk*)(P->ws + P->off_axb[ax]);
        D.ax_nblk[ax] = (int64_t)P->ax_blk[ax].size();
        int64_t ns = 0;
        while (ns < D.ax_nblk[ax] && P->ax_blk[ax][ns].lm <= SHORT_LM) ++ns;
        D.ax_nblk_short[ax] = ns;
        D.ax_vec[ax] = P->ax_vec[ax];
    }
    {
        int64_t np = 0;
        while (np < D.ax_nblk[0] && P->ax_blk[0][np].lm <= CONTIG_PART_LM) ++np;
        D.ax0_nblk_part = np;
    }
    const bool gs = !P->gs_lines.empty();
    D.gs_unit_plane0 = gs ? (const int32_t*)(P->ws + P->off_gsu) : nullptr;
    D.gs_plane_line0 = gs ? (const int64_t*)(P->ws + P->off_gsp) : nullptr;
    D.gs_lines = gs ? (const int32_t*)(P->ws + P->off_gsl) : nullptr;
    D.march = P->march;
    D.march_blk = P->march_blk.empty() ? nullptr : (const MarchBlk*)(P->ws + P->off_march);
    D.march_blk_x = P->march_blk_x.empty() ? nullptr : (const MarchBlk*)(P->ws + P->off_march_x);
    D.n_march = (int64_t)P->march_blk.size();
    D.n_march_x = (int64_t)P->march_blk_x.size();
    D.march_lds = (MARCH_SLOTS * P->march_lp + MARCH_SEG) * (int)P->elem;   // slot ring + V^2 of the planes
    P->bound = true;
    return AMF_OK;
}

}  // namespace

extern "C" {

amf_status amf_plan_bind(amf_plan* P, void* d_ws, uint64_t bytes, void* stream)
{
    if (!P) return fail(AMF_E_INVALID, "null plan");
    if (!d_ws) return fail(AMF_E_INVALID, "null workspace");
    if (bytes < P->ws_bytes) return fail(AMF_E_INVALID, "workspace too small: need " + std::to_string(P->ws_bytes) + " bytes");
    if (((uintptr_t)d_ws & 255u) != 0) return fail(AMF_E_INVALID, "workspace must be 256-byte aligned");
    return bind_impl(P, d_ws, (hipStream_t)stream);
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
    // vectors read or written once: F only 2; stage 1 (W, F(g), out) 3; stage 2 (W, K1, F(g), out)
    // 4; refinement (K^(d), K^(0) in and out) 3; the fused stage operators also write the solved
    // values (one more vector; with the marching operator, of the grids with short axis-1 lines
    // only), the fused refinement writes only those
    double nv = (op == OP_F_PAYOFF || op == OP_F_ZERO) ? 2.0 : (op == OP_STAGE2 ? 4.0 : 3.0);
    if (a.S != nullptr && op != OP_REFINE) nv += P->march ? P->ax_short_frac[0] : 1.0;
    const int kc = op == OP_STAGE1 ? AMF_K_STAGE1 : op == OP_STAGE2 ? AMF_K_STAGE2
                 : op == OP_REFINE ? AMF_K_REFINE : AMF_K_OPERATOR;
    return timed(P, kc, nv * P->vbytes(), s, [&] { return launch_stencil(P->dev, P->prec, op, a, s); });
}

// Both launches (short and long lines) of one directional solve.  Algorithmic bytes: the part's
// share of the vector read and written once (four vectors for the update form).
// part0 = false skips the short-line launch (axis 0 with the marching operator's fused solve).
hipError_t run_sweep(amf_plan* P, int axis, int epi, const SweepArgs& a, hipStream_t s, bool part0 = true)
{
    const bool up = epi == EPI_UPDATE;
    for (int part = part0 ? 0 : 1; part < 2; ++part) {
        const double share = part == 0 ? P->ax_short_frac[axis] : 1.0 - P->ax_short_frac[axis];
        if (share <= 0.0) continue;
        const int kc = axis == 0 ? (part ? AMF_K_SWEEP_CONTIG_LONG : AMF_K_SWEEP_CONTIG)
                     : up ? (part ? AMF_K_SWEEP_UPDATE_LONG : AMF_K_SWEEP_UPDATE)
                          : (part ? AMF_K_SWEEP_STRIDED_LONG : AMF_K_SWEEP_STRIDED);
        const double bytes = (up ? 4.0 : 2.0) * share * (double)P->inner * (double)P->elem;
        hipError_t e = timed(P, kc, bytes, s, [&] { return launch_sweep(P->dev, P->prec, axis, epi, part, a, s); });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Initial data (dis0) in the W = Y - g form: F(g) once (payoff on the lower faces), then W = 0.
hipError_t run_init(amf_plan* P, hipStream_t s)
{
    hipError_t e = timed(P, AMF_K_INIT, P->vbytes(), s, [&] { return launch_payoff(P->dev, P->prec, P->vec(V_A), s); });
    if (e != hipSuccess) return e;
    StencilArgs a{};
    a.X0 = P->vec(V_A);
    a.W = P->vec(V_G);
    a.scale = 1.0;
    a.scale_sel = -1;
    if ((e = run_stencil(P, OP_F_PAYOFF, a, s)) != hipSuccess) return e;
    return timed(P, AMF_K_INIT, P->vbytes(), s, [&] { return launch_fill_zero(P->dev, P->prec, P->vec(V_W), s); });
}

hipError_t run_unit_values(amf_plan* P, double* vals, hipStream_t s)
{
    const double b = (double)P->n_units * (double)(1 << P->d) * (double)P->elem + 8.0 * P->n_units;
    return timed(P, AMF_K_UNIT_VALUES, b, s,
                 [&] { return launch_unit_values(P->dev, P->prec, P->vec(V_W), vals, s); });
}

amf_status one_step(amf_plan* P, int run, hipStream_t s);

// n AMFR-W steps on every unit: one unit-resident launch, or n streaming steps.
amf_status advance(amf_plan* P, int run, int n, hipStream_t s)
{
    if (P->resident) {
        ResArgs a{};
        a.W = P->vec(V_W);
        a.cG = P->vec(V_G);
        a.run = run;
        a.nsteps = n;
        a.a21 = P->sch.a[1 * AMF_MAX_STAGES + 0];
        a.q21 = P->sch.q[1 * AMF_MAX_STAGES + 0];
        a.b1 = P->sch.b[0];
        a.b2 = P->sch.b[1];
        a.lds_len = P->res_lds_len;
        a.tab_len = P->res_tab_len;
        hipError_t e = timed(P, AMF_K_RESIDENT, (2.0 + 2.0 * n) * P->vbytes(), s,
                             [&] { return launch_resident(P->dev, P->prec, a, s); });
        return e == hipSuccess ? AMF_OK : hip_fail(e, "resident");
    }
    for (int i = 0; i < n; ++i) {
        amf_status st = one_step(P, run, s);
        if (st) return st;
    }
    return AMF_OK;
}

// out = (acc ? out : 0) + sum_j c[j] in[j] over whole grid vectors.
hipError_t run_lincomb(amf_plan* P, void* out, bool acc, const void* const* in, const double* c, int n,
                       hipStream_t s)
{
    LinArgs a{};
    a.n = n;
    a.acc = acc ? 1 : 0;
    a.out = out;
    for (int j = 0; j < n; ++j) {
        a.in[j] = in[j];
        a.c[j] = c[j];
    }
    return timed(P, AMF_K_LINCOMB, (n + 1 + (acc ? 1 : 0)) * P->vbytes(), s,
                 [&] { return launch_lincomb(P->dev, P->prec, a, s); });
}

// One step of the s-stage W-method (row-s) on every unit; run selects dt (0: coarse, 1: fine half
// step of the Richardson pair).  Stage r: the right-hand side dt F(Y + sum_j a_rj K_j) + sum_j q_rj K_j
// (one operator launch; for r >= 2 the two sums are formed first), then either the AMF stage of
// eq (amfrw) (chain of directional solves, refinement, second chain) or, for W = P, one
// lower-triangular solve.  The update Y += sum_r b_r K_r is fused into the last directional solve
// (AMF) or is one combination launch (W = P).
amf_status one_step(amf_plan* P, int run, hipStream_t s)
{
    const int d = P->d, S = P->sch.stages;
    const bool lower = P->sch.w_matrix == AMF_W_LOWER;
    const int sel_dt = CST_RUN + 3 * run, sel_th = sel_dt + 2;
    void *Wv = P->vec(V_W), *A = P->vec(V_A), *B = P->vec(V_B), *G = P->vec(V_G);
    auto K = [&](int r) { return P->vec(V_K0 + r); };
    auto ca = [&](int r, int j) { return P->sch.a[r * AMF_MAX_STAGES + j]; };
    auto cq = [&](int r, int j) { return P->sch.q[r * AMF_MAX_STAGES + j]; };
    const bool fuse = P->fuse0 != 0 && !lower;
    // the marching operator fuses the axis-1 solve of the units with short axis-1 lines only: the
    // chain then starts at axis 0 with the long-line launch, in place over the operator's output
    const bool mfuse = fuse && P->march;
    const int first = fuse && !mfuse ? 1 : 0;
    hipError_t e;
    // (I - nu dt A_1) .. (I - nu dt A_d) applied in axis order from axis `first` (1 when the operator
    // launch already solved axis 0); the first solve reads `in`, the others work in place on `dst`;
    // with `update` the last solve ends in W += b1 U + b2 x
    auto chain = [&](const void* in, void* dst, bool update, const void* U, double b1, double b2) -> hipError_t {
        for (int ax = first; ax < d; ++ax) {
            SweepArgs a{};
            a.in = ax == first ? in : dst;
            a.out = dst;
            a.run = run;
            int epi = EPI_STORE;
            if (update && ax == d - 1) {
                epi = EPI_UPDATE;
                a.out = Wv;
                a.K1 = U;
                a.b1 = b1;
                a.b2 = b2;
            }
            hipError_t err = run_sweep(P, ax, epi, a, s, !(mfuse && ax == 0));
            if (err != hipSuccess) return err;
        }
        return hipSuccess;
    };
    for (int r = 0; r < S; ++r) {
        const bool last = r == S - 1;
        // ---- right-hand side K^(0) -> A (fused: and its axis-0 solve -> B)
        StencilArgs st{};
        st.X0 = Wv;
        st.cG = G;
        st.W = A;
        st.S = fuse ? B : nullptr;
        st.run = run;
        st.scale_sel = sel_dt;
        int op = OP_STAGE1;
        if (r == 1) {
            op = OP_STAGE2;
            st.X1 = K(0);
            st.X2 = K(0);
            st.a = ca(1, 0);
            st.q = cq(1, 0);
        } else if (r >= 2) {
            const void* in[AMF_MAX_STAGES];
            double c[AMF_MAX_STAGES];
            for (int j = 0; j < r; ++j) {
                in[j] = K(j);
                c[j] = ca(r, j);
            }
            if ((e = run_lincomb(P, P->vec(P->v_z), false, in, c, r, s)) != hipSuccess) return hip_fail(e, "lincomb");
            for (int j = 0; j < r; ++j) c[j] = cq(r, j);
            if ((e = run_lincomb(P, P->vec(P->v_q), false, in, c, r, s)) != hipSuccess) return hip_fail(e, "lincomb");
            op = OP_STAGE2;
            st.X1 = P->vec(P->v_z);
            st.X2 = P->vec(P->v_q);
            st.a = 1.0;
            st.q = 1.0;
        }
        if ((e = run_stencil(P, op, st, s)) != hipSuccess) return hip_fail(e, "stencil");
        if (lower) {
            // (I - theta dt P) K_r = K^(0); the last stage's K stays in A
            LowerArgs la{};
            la.rhs = A;
            la.x = last ? A : K(r);
            la.run = run;
            e = timed(P, AMF_K_LOWER, 2.0 * P->vbytes(), s, [&] { return launch_lower(P->dev, P->prec, la, s); });
            if (e != hipSuccess) return hip_fail(e, "lower solve");
            if (last) {
                const void* in[AMF_MAX_STAGES];
                double c[AMF_MAX_STAGES];
                for (int j = 0; j < S - 1; ++j) {
                    in[j] = K(j);
                    c[j] = P->sch.b[j];
                }
                in[S - 1] = A;
                c[S - 1] = P->sch.b[S - 1];
                if ((e = run_lincomb(P, Wv, true, in, c, S, s)) != hipSuccess) return hip_fail(e, "lincomb");
            }
            continue;
        }
        if ((e = chain(fuse && !mfuse ? B : A, B, false, nullptr, 0.0, 0.0)) != hipSuccess) return hip_fail(e, "sweep");
        // Khat^(0) = 2 K^(0) - K^(d) + theta dt F(K^(d)) -> A; fused: its axis-0 solve -> dst (the last
        // stage's goes back over A, which no other block reads)
        void* dst = last ? (fuse ? A : B) : K(r);
        st = StencilArgs{};
        st.X0 = B;
        st.W = A;
        st.S = fuse ? (last ? A : dst) : nullptr;
        st.run = run;
        st.scale_sel = sel_th;
        if ((e = run_stencil(P, OP_REFINE, st, s)) != hipSuccess) return hip_fail(e, "stencil");
        if (!last) {
            if ((e = chain(fuse && !mfuse ? dst : A, dst, false, nullptr, 0.0, 0.0)) != hipSuccess) return hip_fail(e, "sweep");
            continue;
        }
        // the last chain ends in W += sum_{j<s} b_j K_j + b_s K_s: for s = 2 the sum is b_1 K_1
        const void* U = nullptr;
        double b1 = 0.0;
        if (S == 2) {
            U = K(0);
            b1 = P->sch.b[0];
        } else if (S > 2) {
            const void* in[AMF_MAX_STAGES];
            double c[AMF_MAX_STAGES];
            for (int j = 0; j < S - 1; ++j) {
                in[j] = K(j);
                c[j] = P->sch.b[j];
            }
            if ((e = run_lincomb(P, P->vec(P->v_z), false, in, c, S - 1, s)) != hipSuccess) return hip_fail(e, "lincomb");
            U = P->vec(P->v_z);
            b1 = 1.0;
        } else {
            U = G;              // s = 1: nothing to add (b1 = 0); any vector of the plan is a valid read
        }
        if ((e = chain(A, dst, true, U, b1, P->sch.b[S - 1])) != hipSuccess) return hip_fail(e, "sweep");
    }
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
    // the state no longer belongs to a completed Richardson pair: combine without extrapolation
    P->have_coarse = false;
    return advance(P, 0, n, (hipStream_t)stream);
}

namespace {

// The whole solve (initial data, n_steps steps, and the fine run of a Richardson pair) on stream s.
amf_status solve_body(amf_plan* P, hipStream_t s)
{
    amf_status st;
    hipError_t e = run_init(P, s);
    if (e != hipSuccess) return hip_fail(e, "init");
    if ((st = advance(P, 0, P->steps, s))) return st;
    if (P->richardson) {
        e = run_unit_values(P, (double*)(P->ws + P->off_valsc), s);
        if (e != hipSuccess) return hip_fail(e, "unit values");
        if ((e = timed(P, AMF_K_INIT, P->vbytes(), s, [&] { return launch_fill_zero(P->dev, P->prec, P->vec(V_W), s); })) != hipSuccess)
            return hip_fail(e, "init");
        if ((st = advance(P, 1, 2 * P->steps, s))) return st;
    }
    return AMF_OK;
}

amf_status capture_graph(amf_plan* P)
{
    hipError_t e;
    if (!P->cap_stream && (e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreateWithFlags");
    if ((e = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
    amf_status st = solve_body(P, P->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(P->cap_stream, &g);
    if (st != AMF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t gx = nullptr;
    if ((e = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    P->graph = g;
    P->graph_exec = gx;
    P->graph_valid = true;
    return AMF_OK;
}

}  // namespace

amf_status amf_graph_enable(amf_plan* P, int32_t on)
{
    if (!P) return fail(AMF_E_INVALID, "null plan");
    if (on != 0 && on != 1) return fail(AMF_E_INVALID, "on must be 0 or 1");
    if (!on) P->drop_graph();
    P->graph_on = on != 0;
    return AMF_OK;
}

amf_status amf_solve(amf_plan* P, void* stream)
{
    amf_status st = check_bound(P);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (P->graph_on && !P->prof) {
        if (!P->graph_valid && (st = capture_graph(P))) return st;
        hipError_t e = hipGraphLaunch(P->graph_exec, s);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    } else {
        if ((st = solve_body(P, s))) return st;
    }
    P->initialised = true;
    P->have_coarse = P->richardson != 0;
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

amf_status amf_combine_checked(amf_plan* P, double* d_prices, void* stream)
{
    amf_status st = amf_combine(P, d_prices, stream);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    int32_t* flag = (int32_t*)(P->ws + P->off_flag);
    hipError_t e = launch_first_nonfinite(d_prices, P->n_probs, flag, s);
    if (e != hipSuccess) return hip_fail(e, "check prices");
    int32_t bad = -1;
    if ((e = hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (bad >= 0) return fail(AMF_E_NUMERIC, "non-finite price of problem " + std::to_string(bad) +
                                              " (an unstable configuration: raise nu or the step count)");
    return AMF_OK;
}

amf_status amf_price_or_fallback(amf_mlp* mlp, amf_plan* P, const float* d_x, float tol, float abs_floor,
                                 double* d_prices, int32_t* d_used_solver, void* stream)
{
    amf_status st = check_bound(P);
    if (st) return st;
    if (!mlp || !d_x || !d_prices || !d_used_solver) return fail(AMF_E_INVALID, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const int n = P->n_probs;
    // 1. network prices and routing flags on the device
    if ((st = mlp_route(mlp, d_x, n, tol, abs_floor, d_prices, d_used_solver, s))) return fail(st, mlp_error());
    std::vector<int32_t> used((size_t)n), idx;
    hipError_t e = hipMemcpyAsync(used.data(), d_used_solver, (size_t)n * 4, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (int i = 0; i < n; ++i)
        if (used[(size_t)i]) idx.push_back(i);
    const int k = (int)idx.size();
    // 2. the routed requests through the solver
    if (k == n) {
        if ((st = amf_solve(P, stream)) || (st = amf_combine(P, d_prices, stream))) return st;
    } else if (k > 0) {
        std::vector<amf_problem> sub((size_t)k);
        for (int j = 0; j < k; ++j) sub[(size_t)j] = P->probs[(size_t)idx[(size_t)j]];
        amf_plan* Q = nullptr;
        if ((st = amf_plan_create(sub.data(), k, &P->grid, &P->sch, (amf_precision)P->prec, P->steps,
                                  P->richardson, &Q)))
            return st;
        std::unique_ptr<amf_plan> hold(Q);
        // a subset of the parent's units packs into no more space than the parent's own layout
        if (Q->core_bytes > P->core_bytes) return fail(AMF_E_STATE, "fallback plan does not fit the workspace");
        Q->stencil_r = P->stencil_r;          // same grids per problem: the parent's schedule is valid
        Q->xcd = P->xcd;
        Q->fuse0 = P->fuse0;
        Q->resident = P->resident && Q->res_ok;
        double* stage = (double*)(P->ws + P->off_fb);
        int32_t* sidx = (int32_t*)(P->ws + P->off_fb + (size_t)n * sizeof(double));
        st = bind_impl(Q, P->ws, s);           // overwrites the parent's tables and state
        if (!st) st = amf_solve(Q, stream);
        if (!st) st = amf_combine(Q, stage, stream);
        if (!st) st = upload(sidx, idx.data(), (size_t)k * 4, s);
        if (!st && (e = launch_scatter(stage, sidx, k, d_prices, s)) != hipSuccess) st = hip_fail(e, "scatter");
        if (!st && (e = hipStreamSynchronize(s)) != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
        // the parent's tables back in place (its state is gone: amf_solve before reading it)
        amf_status st2 = bind_impl(P, P->ws, s);
        if (st) return st;
        if (st2) return st2;
    }
    // 3. the failure signal of an unstable configuration
    int32_t* flag = (int32_t*)(P->ws + P->off_flag);
    if ((e = launch_first_nonfinite(d_prices, n, flag, s)) != hipSuccess) return hip_fail(e, "check prices");
    int32_t bad = -1;
    if ((e = hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (bad >= 0) return fail(AMF_E_NUMERIC, "non-finite price of request " + std::to_string(bad));
    return AMF_OK;
}

}  // extern "C"

namespace {

// Workspace of amf_solve_static: a file-scope device array, one copy per GPU the library runs on,
// held until the process ends.  Host code never uses its name as an address: the device address
// comes from hipGetSymbolAddress, once per device (with that device current), kept in g_static.
constexpr size_t STATIC_BYTES = AMF_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[STATIC_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_static_mu;
void* g_static[MAX_DEVICES] = {};

amf_status static_workspace(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(AMF_E_UNSUPPORTED, "device index beyond the static workspace table");
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress");
        if (!ptr || ((uintptr_t)ptr & 255u)) return fail(AMF_E_HIP, "static workspace address is not 256-byte aligned");
        g_static[dev] = ptr;
    }
    *out = g_static[dev];
    return AMF_OK;
}

}  // namespace

extern "C" {

amf_status amf_solve_static(amf_plan* P, double* d_prices, void* stream)
{
    if (!P || !d_prices) return fail(AMF_E_INVALID, "null argument");
    if (P->core_bytes > STATIC_BYTES)
        return fail(AMF_E_INVALID, "plan needs " + std::to_string(P->core_bytes) + " bytes of workspace; the static "
                                   "workspace holds " + std::to_string(STATIC_BYTES));
    void* ws = nullptr;
    amf_status st = static_workspace(&ws);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    // the plan's own binding (if any) is left as it was: its workspace is not touched
    char* const saved_ws = P->ws;
    const DevPlan saved_dev = P->dev;
    const bool saved_bound = P->bound, saved_init = P->initialised, saved_coarse = P->have_coarse;
    st = bind_impl(P, ws, s);                          // tables into the static workspace
    if (!st) st = solve_body(P, s);                    // eager launches: nothing is captured
    if (!st) {
        P->have_coarse = P->richardson != 0;
        st = amf_combine(P, d_prices, stream);
    }
    P->ws = saved_ws;                                  // kernels already hold their arguments
    P->dev = saved_dev;
    P->bound = saved_bound;
    P->initialised = saved_init;
    P->have_coarse = saved_coarse;
    return st;
}

amf_status amf_state_read(amf_plan* P, void* d_out, void* stream)
{
    amf_status st = check_bound(P);
    if (st) return st;
    if (!d_out) return fail(AMF_E_INVALID, "null output");
    hipError_t e = launch_state_read(P->dev, P->prec, P->vec(V_W), d_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "state read");
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
    a.run = 0;
    for (int part = 0; part < 2; ++part) {
        hipError_t e = launch_sweep(P->dev, P->prec, axis, EPI_STORE, part, a, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "sweep");
    }
    return AMF_OK;
}

amf_status amf_schedule_get(const amf_plan* P, amf_schedule* out)
{
    if (!P || !out) return fail(AMF_E_INVALID, "null argument");
    out->struct_size = sizeof(amf_schedule);
    out->stencil_nodes = P->stencil_r;
    out->xcd_remap = P->xcd;
    out->max_stencil_nodes = 8;
    out->resident = P->resident;
    out->resident_available = P->res_ok ? 1 : 0;
    out->fuse_axis0 = P->fuse0;
    out->fuse_max_axis0 = P->max_m0;
    out->march = P->march;
    out->march_available = P->march_blk.empty() ? 0 : 1;
    return AMF_OK;
}

amf_status amf_schedule_set(amf_plan* P, const amf_schedule* sc)
{
    if (!P || !sc || sc->struct_size != sizeof(amf_schedule)) return fail(AMF_E_INVALID, "bad amf_schedule");
    const int r = sc->stencil_nodes;
    if (r != 1 && r != 2 && r != 4 && r != 8) return fail(AMF_E_INVALID, "stencil_nodes must be 1, 2, 4 or 8");
    if (sc->xcd_remap < 0 || sc->xcd_remap > 2) return fail(AMF_E_INVALID, "xcd_remap must be 0, 1 or 2");
    if (sc->resident != 0 && sc->resident != 1) return fail(AMF_E_INVALID, "resident must be 0 or 1");
    if (sc->resident && !P->res_ok) return fail(AMF_E_INVALID, "a unit exceeds the unit-resident size limit");
    if (sc->fuse_axis0 != 0 && sc->fuse_axis0 != 1) return fail(AMF_E_INVALID, "fuse_axis0 must be 0 or 1");
    if (sc->fuse_axis0 && P->sch.w_matrix != AMF_W_AMF)
        return fail(AMF_E_INVALID, "fuse_axis0 applies to the AMF W only");
    if (sc->march != 0 && sc->march != 1) return fail(AMF_E_INVALID, "march must be 0 or 1");
    if (sc->march && P->march_blk.empty()) return fail(AMF_E_INVALID, "the marching operator needs d <= 4");
    if (sc->fuse_axis0 && !sc->march &&
        (r < 2 || r > P->min_m0 || NODE_BLOCK * r < P->max_m0 || P->max_m0 > (1 << CONTIG_PART_LM)))
        return fail(AMF_E_INVALID, "fuse_axis0 needs 2 <= stencil_nodes <= the shortest axis-1 line and 256 * "
                                   "stencil_nodes >= the longest one (at most 1024 points)");
    if (sc->fuse_axis0 && sc->march && P->max_m0 > (1 << CONTIG_PART_LM))
        return fail(AMF_E_INVALID, "fuse_axis0 with the marching operator needs axis-1 lines of at most 1024 points");
    if (r != P->stencil_r || sc->xcd_remap != P->xcd || sc->resident != P->resident || sc->fuse_axis0 != P->fuse0 ||
        sc->march != P->march)
        P->drop_graph();
    P->march = sc->march;
    P->dev.march = sc->march;
    P->resident = sc->resident;
    P->fuse0 = sc->fuse_axis0;
    P->stencil_r = r;
    P->xcd = sc->xcd_remap;
    P->dev.stencil_r = r;
    P->dev.xcd = P->xcd;
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
