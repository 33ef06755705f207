// Internal declarations shared by the host plan code and the gfx950 kernels of libamfrw.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "amfrw.h"
#include "amfrw_consts.h"
#include "amfrw_march.h"

namespace amf {

constexpr int NODE_BLOCK = 256;    // threads per block of the per-node kernels
constexpr int WAVE = 64;           // lanes of a wavefront
constexpr int LINE_BLOCK = 256;    // threads per block of the sweep kernels
constexpr int PAIR_LM = 2;         // short strided lines of at most 2^PAIR_LM points: two line slots per thread
constexpr int UNIT_ALIGN = 64;     // unit offsets are multiples of 64 elements
constexpr int SEG = 16;            // rows per lane in the partitioned solve of long contiguous lines
// Longer strided lines: seg_rows consecutive rows per thread (one line: 8 in FP64, 32 in FP32;
// measured on the d = 4 workload), M/seg_rows threads per line, blocks of SEG_BLOCK threads
// (SEG_BLOCK*seg_rows/M line slots each), up to SEG_BLOCK*seg_rows rows; beyond that one block per
// line walks it in chunks of SEG_BLOCK*seg_rows rows.
constexpr int SSEG_F64 = 8;
constexpr int SSEG_F32 = 32;
constexpr int SEG_BLOCK = 512;
// rows per thread by element size and by lines per thread (vec > 1: vec adjacent lines carried as
// one vector: 128 bytes of line data per thread)
constexpr int seg_rows(int elem, int vec) { return vec > 1 ? 128 / (vec * elem) : (elem == 8 ? SSEG_F64 : SSEG_F32); }
// log2 of the longest line the segmented solver takes: SEG_BLOCK * seg_rows rows
constexpr int seg_max_lm(int elem, int vec)
{
    int r = SEG_BLOCK * seg_rows(elem, vec), l = 0;
    while (r > 1) { r >>= 1; ++l; }
    return l;
}
constexpr int NXCD = 8;            // MI355X: 8 XCDs, each with its own L2
// index of the node-block table for R nodes per thread (R = 1, 2, 4, 8)
constexpr int r_index(int R) { return R == 8 ? 3 : R == 4 ? 2 : R == 2 ? 1 : 0; }
// Default nodes per thread of the time-loop operator, by precision (limited by each unit's M_0);
// a plan's schedule may override it (the autotuner picks among 1, 2, 4, 8).
constexpr int STENCIL_R_F64 = 4;
constexpr int STENCIL_R_F32 = 4;
// Contiguous (axis 0) lines up to 2^CONTIG_REG_LM are solved by one thread; longer ones up to
// 2^CONTIG_PART_LM by SEG-row segments on M/SEG cooperating lanes of one wavefront; longer still by
// the segmented block solver of the strided axes (stride 1, tabulated factors).
constexpr int CONTIG_REG_LM = 4;
constexpr int CONTIG_PART_LM = 10;
// Sweep launches are split by line length: classes up to 2^SHORT_LM and longer ones, so that
// short lines are not held to the register allocation of the long-line code.
constexpr int SHORT_LM = 4;


// One unit = one (problem, component grid) pair.  Inner nodes only, axis 0 fastest.
struct alignas(16) UnitDev {
    int64_t off;          // element offset of the unit in every grid vector (multiple of UNIT_ALIGN)
    int32_t prob;         // problem index
    int32_t lsum;         // sum of levels = log2(#inner points)
    int8_t lv[MAXD];      // log2 M_i
    int8_t pad_[2];
    int32_t tab[MAXD];    // offset of the coefficient block of (prob, axis i, lv_i) in the tables
    int32_t fac[MAXD];    // offset of the Thomas factor block of (prob, axis i, lv_i, lv_V), run 0
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
    int32_t dirichlet;    // 1: the upper faces of the rate axes hold the payoff (eq bound1_0)
    int32_t pad_[3];
};

// Whether a node with rate-axis index j on an axis of M intervals is boundary data: the upper face
// of a rate axis under the Dirichlet conditions of eq (bound1_0).
__host__ __device__ __forceinline__ bool dir_face(int dirichlet, int j, int M) { return dirichlet && j == M; }

// A block of the sweep along one axis: lines [line_start, line_end) of the axis' line list, all
// of length 2^lm; k_start indexes the axis' unit list at line_start; vec: adjacent lines per
// thread of the short-line sweep (1, or 16 B / element when all the block's units allow it);
// slots: line slots per thread of the short-line sweep (2 for lines of at most 2^PAIR_LM points on
// the axes 2..N-1, the second LINE_BLOCK slots after the first; else 1).
struct alignas(16) SweepBlk {
    int64_t line_start;
    int64_t line_end;
    int32_t k_start;
    int32_t lm;
    int32_t vec;
    int32_t slots;
};

// A block of the streaming operator with R consecutive axis-1 nodes per thread, over one run of
// consecutive units of the same line class: nodes g0 + t R, t < NODE_BLOCK, below gend.
struct alignas(8) VecBlk {
    int64_t g0, gend;
    int32_t unit;         // the unit containing g0 (or whose padding holds it)
    int32_t pad_;
};
// lists: units with M_1 == 1, 2, 4 (ids 0..2) and with M_1 >= 1, 2, 4, 8 (ids 3..6)
constexpr int VB_LISTS = 7;
constexpr int vb_exact(int R) { return R == 4 ? 2 : R == 2 ? 1 : 0; }
constexpr int vb_atleast(int R) { return 3 + (R == 8 ? 3 : R == 4 ? 2 : R == 2 ? 1 : 0); }

// Device view of a bound plan (pointers into the workspace).
struct DevPlan {
    int d;
    int n_units;
    int n_probs;
    int64_t total;               // elements per grid vector (inner points + alignment padding)
    const UnitDev* units;        // n_units + 1 (sentinel off = total)
    const ProbDev* probs;
    const void* tab;             // coefficient tables, plan precision
    const void* fac;             // Thomas factor tables (inv, a*inv, c'), plan precision
    int64_t fac_run_stride;      // elements between the run-0 and run-1 factor tables
    const int32_t* blk_unit;     // per node block: first unit
    int64_t n_node_blocks;
    int stencil_r;               // nodes per thread of the time-loop operator (1, 2, 4 or 8)
    int xcd;                     // 1: XCD-aware block remapping
    const int32_t* blk_unit_r[4];   // per block of NODE_BLOCK * R nodes (R = 1, 2, 4, 8): first unit
    int64_t n_blocks_r[4];
    // operator blocks by axis-1 line class (units with M_1 = 1, 2, 4; M_1 >= 1, 2, 4, 8)
    const VecBlk* vblk;
    int64_t vblk_off[VB_LISTS], vblk_n[VB_LISTS];
    const int32_t* ax_units[MAXD];     // per axis: units ordered by M_axis
    const int64_t* ax_line_off[MAXD];  // per axis: first line of each listed unit (+ sentinel)
    const SweepBlk* ax_blk[MAXD];
    int64_t ax_nblk[MAXD];
    int64_t ax_nblk_short[MAXD];       // leading blocks with lm <= SHORT_LM
    int64_t ax0_nblk_part;             // axis 0: leading blocks with lm <= CONTIG_PART_LM
    int ax_vec[MAXD];                  // long strided lines: 16-byte vectors of adjacent lines per slot
    // W = P solves: unit u's hyperplanes are [gs_unit_plane0[u], gs_unit_plane0[u+1]); plane p holds
    // the axis-0 lines gs_lines[gs_plane_line0[p] .. gs_plane_line0[p+1]) (line id = loc >> lv_0)
    const int32_t* gs_unit_plane0;
    const int64_t* gs_plane_line0;
    const int32_t* gs_lines;
    // marching (plane-tiled) operator, d <= 4: blocks and dynamic LDS bytes per block
    int march;                         // 1: the time-loop operators use the marching kernel
    const MarchBlk* march_blk;         // unit by unit
    const MarchBlk* march_blk_x;       // grouped per XCD (used when xcd != 0)
    int64_t n_march, n_march_x;
    int march_lds;
};


struct StencilArgs {
    const void* X0;
    const void* X1;
    const void* X2;       // OP_STAGE2: the vector q multiplies (X1 when null)
    const void* cG;
    void* W;
    void* S;              // non-null: fused axis-0 solve, solved values written here
    double a, q;          // OP_STAGE2 coefficients
    double scale;         // explicit scale when scale_sel < 0
    int scale_sel;        // else index into the per-problem constant block
    int run;              // factor tables of the fused solve: 0 coarse, 1 fine (Richardson) step
};

enum SweepEpi : int { EPI_STORE = 0, EPI_UPDATE = 1 };

struct SweepArgs {
    const void* in;
    void* out;            // EPI_STORE target; EPI_UPDATE: the solution W (updated in place)
    const void* K1;       // EPI_UPDATE: first stage
    double b1, b2;        // EPI_UPDATE: W += b1 K1 + b2 x
    int run;              // 0 coarse, 1 fine (Richardson)
};

// Unit-resident schedule: one workgroup of RES_BLOCK threads per unit, the whole time loop in LDS.
constexpr int RES_BLOCK = 128;
constexpr int RES_MAX_LSUM_F32 = 11;   // units up to 2048 points (4 FP32 vectors: at most 40 KB)
constexpr int RES_MAX_LSUM_F64 = 10;   // units up to 1024 points (4 FP64 vectors: at most 40 KB)
// Pitch of the axis-1 rows of a resident unit in LDS: one padding element per row of 4 or more
// nodes, so that the lanes of an axis-1 line solve (one row each) fall on distinct banks.
__host__ __device__ __forceinline__ int res_pitch(int m0) { return m0 >= 4 ? m0 + 1 : m0; }

struct ResArgs {
    void* W;              // solution W (global), read at entry and written at exit
    const void* cG;       // F(g) (global)
    int run, nsteps;
    double a21, q21, b1, b2;
    int lds_len;          // elements per LDS vector: the largest unit's rows at res_pitch(M_1)
    int tab_len;          // elements of the largest unit's 1-D coefficient tables
};

// out = (acc ? out : 0) + sum_{j < n} c_j in_j over every element of a grid vector.
constexpr int LIN_MAX = 7;
struct LinArgs {
    const void* in[LIN_MAX];
    double c[LIN_MAX];
    int n;
    int acc;
    void* out;
};

// (I - theta dt P) x = rhs on every unit, P the lower triangle of the Sketch-1 matrix: one workgroup
// per unit walks its hyperplanes sum_{i>=1} i (j_i - 1) = const of axis-0 lines; x may overwrite rhs.
constexpr int LOWER_BLOCK = 256;
struct LowerArgs {
    const void* rhs;
    void* x;
    int run;              // 0 coarse, 1 fine (Richardson): theta dt from the constant block
};

// Kernel launchers (amfrw_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_lincomb(const DevPlan& P, int prec, const LinArgs& a, hipStream_t s);
// flag = index of the first non-finite entry of p[0..n), or -1
hipError_t launch_first_nonfinite(const double* p, int n, int32_t* flag, hipStream_t s);
// dst[idx[i]] = src[i], i < n
hipError_t launch_scatter(const double* src, const int32_t* idx, int n, double* dst, hipStream_t s);

// Surrogate router (amfrw_mlp.hip): network prices and solver-routing flags for n requests.
amf_status mlp_route(amf_mlp* N, const float* d_x, int64_t n, float tol, float abs_floor, double* d_prices,
                     int32_t* d_used, hipStream_t s);
const char* mlp_error();
hipError_t launch_lower(const DevPlan& P, int prec, const LowerArgs& a, hipStream_t s);
hipError_t launch_resident(const DevPlan& P, int prec, const ResArgs& a, hipStream_t s);
hipError_t launch_payoff(const DevPlan& P, int prec, void* Y, hipStream_t s);
hipError_t launch_fill_zero(const DevPlan& P, int prec, void* Y, hipStream_t s);
hipError_t launch_state_read(const DevPlan& P, int prec, const void* W, void* Y, hipStream_t s);
hipError_t launch_stencil(const DevPlan& P, int prec, int op, const StencilArgs& a, hipStream_t s);
// part 0: lines up to 2^SHORT_LM points; part 1: longer lines.
hipError_t launch_sweep(const DevPlan& P, int prec, int axis, int epi, int part, const SweepArgs& a,
                        hipStream_t s);
hipError_t launch_unit_values(const DevPlan& P, int prec, const void* W, double* vals,
                              hipStream_t s);
hipError_t launch_combine(const DevPlan& P, const double* coef, const double* vals,
                          const double* vals_coarse, double* prices, hipStream_t s);

}  // namespace amf
