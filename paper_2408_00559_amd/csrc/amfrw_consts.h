// Plain layout constants of libamfrw shared by the host plan code, the gfx950 kernels and the host
// emulation of the marching operator (no HIP types here).
#pragma once

namespace amf {

constexpr int MAXD = 6;            // kernels are instantiated for d = 2..6
constexpr int MAX_LEVEL = 20;      // per-axis level: at most 2^20 inner points on one axis

// Per-problem constants in the plan precision, at ProbDev::cst inside the table array.
enum CstIndex : int {
    CST_RHO = 0,                     // rho_ik between rates i, k (MAXD x MAXD, row-major)
    CST_SPHI = MAXD * MAXD,          // sigma * phi_i
    CST_RUN = CST_SPHI + MAXD,       // per run (coarse, fine): dt, nu dt, theta dt
    CST_SIZE = CST_RUN + 6
};

// Stencil operation selector.  Solution vectors are stored as W = Y - g (zero on every lower face);
// cG = F(g) is computed once per solve with the payoff on the lower faces.
enum StencilOp : int {
    OP_F_PAYOFF = 0,   // W = s F(X0), lower faces = payoff
    OP_F_ZERO = 1,     // W = s F(X0), lower faces = 0
    OP_STAGE1 = 2,     // W = s (F(X0) + cG)                  (first stage, X0 = W_n)
    OP_STAGE2 = 3,     // W = s (F(X0 + a X1) + cG) + q X2    (later stages; AMFR-W2: X1 = X2 = K_1)
    OP_REFINE = 4      // W = 2 W - X0 + s F(X0)              (refinement of eq amfrw)
};

}  // namespace amf
