// Internal declarations shared by the host plan code and the gfx950 kernels of libamfrw.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace amf {

constexpr int MAXD = 6;            // kernels are instantiated for d = 2..6
constexpr int NODE_BLOCK = 256;    // threads per block of the per-node kernels
constexpr int LINE_BLOCK = 256;    // lines per block of the sweep kernels
constexpr int REG_LM_F64 = 5;      // lines up to 2^5 points keep their Thomas factors in VGPRs (FP64)
constexpr int REG_LM_F32 = 6;      // ... up to 2^6 points in FP32

// Per-problem constants in the plan precision, at ProbDev::cst inside the table array.
enum CstIndex : int {
    CST_RHO = 0,                     // rho_ik between rates i, k (MAXD x MAXD, row-major)
    CST_SPHI = MAXD * MAXD,          // sigma * phi_i
    CST_RUN = CST_SPHI + MAXD,       // per run (coarse, fine): dt, nu dt, theta dt
    CST_SIZE = CST_RUN + 6
};

// One unit = one (problem, component grid) pair.  Inner nodes only, axis 0 fastest.
struct alignas(16) UnitDev {
    int64_t off;          // element offset of the unit in every grid vector
    int32_t prob;         // problem index
    int32_t lsum;         // sum of levels = log2(#inner points)
    int8_t lv[MAXD];      // log2 M_i
    int8_t pad_[2];
    int32_t tab[MAXD];    // offset (elements) of the coefficient block of (prob, axis i, lv_i)
};

// Per-problem data in FP64 (payoff, interpolation, combination).
struct alignas(16) ProbDev {
    double xmax[MAXD];
    double xeval[MAXD];
    double tau[MAXD];
    double K;
    double discount;
    int32_t payoff;       // 0 caplet, 1 swaption
    int32_t cst;          // offset of the CstIndex block in the table array
    int32_t unit_begin;   // units of this problem are [unit_begin, unit_end)
    int32_t unit_end;
};

// A block of the sweep along one axis: lines [line_start, line_end) of the axis' line list, all
// of length 2^lm; k_start indexes the axis' unit list at line_start.
struct alignas(16) SweepBlk {
    int64_t line_start;
    int64_t line_end;
    int32_t k_start;
    int32_t lm;
};

// Device view of a bound plan (pointers into the workspace).
struct DevPlan {
    int d;
    int n_units;
    int n_probs;
    int64_t total;               // inner points over all units
    const UnitDev* units;        // n_units + 1 (sentinel off = total)
    const ProbDev* probs;
    const void* tab;             // coefficient tables, plan precision
    const int32_t* blk_unit;     // per node block: first unit
    int64_t n_node_blocks;
    const int32_t* ax_units[MAXD];     // per axis: units ordered by M_axis
    const int64_t* ax_line_off[MAXD];  // per axis: first line of each listed unit (+ sentinel)
    const SweepBlk* ax_blk[MAXD];
    int64_t ax_nblk[MAXD];
};

// Stencil operation selector.
enum StencilOp : int {
    OP_F_PAYOFF = 0,   // W = s F(X0), lower faces = payoff
    OP_F_ZERO = 1,     // W = s F(X0), lower faces = 0
    OP_STAGE = 2,      // W = s F(X0 + a X1) + q X1, lower faces = payoff
    OP_REFINE = 3      // W = 2 W - X0 + s F(X0), lower faces = 0
};

struct StencilArgs {
    const void* X0;
    const void* X1;
    void* W;
    double a, q;          // OP_STAGE coefficients
    double scale;         // explicit scale when scale_sel < 0
    int scale_sel;        // else index into the per-problem constant block
};

enum SweepEpi : int { EPI_STORE = 0, EPI_UPDATE = 1 };

struct SweepArgs {
    const void* in;
    void* out;            // EPI_STORE target; EPI_UPDATE: the solution Y (updated in place)
    void* cbuf;           // scratch vector for long lines
    const void* K1;       // EPI_UPDATE: first stage
    double b1, b2;        // EPI_UPDATE: Y += b1 K1 + b2 x
    int nudt_sel;         // index into the per-problem constant block
};

// Kernel launchers (amfrw_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_init(const DevPlan& P, int prec, void* Y, hipStream_t s);
hipError_t launch_stencil(const DevPlan& P, int prec, int op, const StencilArgs& a, hipStream_t s);
hipError_t launch_sweep(const DevPlan& P, int prec, int axis, int epi, const SweepArgs& a,
                        hipStream_t s);
hipError_t launch_unit_values(const DevPlan& P, int prec, const void* Y, double* vals,
                              hipStream_t s);
hipError_t launch_combine(const DevPlan& P, const double* coef, const double* vals,
                          const double* vals_coarse, double* prices, hipStream_t s);

}  // namespace amf
