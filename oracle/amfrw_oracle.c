/*
 * amfrw_oracle.c -- plain, slow FP64 CPU reference ("oracle") for the AMFR-W time stepping and the
 * (modified) sparse-grid combination technique of Lopez-Salas, Perez-Rodriguez and Vazquez,
 * "AMFR-W numerical methods for solving high dimensional SABR/LIBOR PDE models" (arXiv 2408.00559).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or helper with the GPU path.
 *
 * Everything is IEEE binary64.  Every routine follows the paper's own statement of the method in the
 * paper's order and notation; nothing is blocked, fused, tabulated or reordered beyond what the
 * paper states.  Storage is the paper's full-grid vector Y of Section 3: all prod(M_i+1) nodes,
 * numbered by the bijection theta_0 (axis 1 fastest), with the lower-face ("Outer") entries holding
 * the payoff for solution vectors and 0 for stage increments.
 *
 * Axes are 0-based here: axis k = 0..N-1 is the paper's F_{k+1}; axis N-1 is the volatility V = F_N.
 * Forward-rate parameters (alpha, phi, tau, rho) are indexed by rate 0..N-2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXD 8
#define ORC_MAXS 6

/* Model selector.  SABR_LMM: the PDE (mmNd) with coefficients (coef_diff), (coef_mix), (coef_adv).
 * CONST_COEF: a constant-coefficient correlated diffusion u_t = sum_ik D_ik u_ik + sum_i c_i u_i used
 * only as a closed-form pin (same Sketch-1 stencil and boundary treatment, constant coefficients). */
enum { ORC_SABR_LMM = 0, ORC_CONST_COEF = 1 };
/* Payoffs: caplet tau_1 (F_1-K)^+ (Section 2), swaption of Section 2 (the max{...} formula), and a
 * Gaussian bump exp(-|x-c|^2/(2w^2)) for the closed-form pin. */
enum { ORC_CAPLET = 0, ORC_SWAPTION = 1, ORC_GAUSSIAN = 2 };
/* Boundary conditions on the upper faces F_j = F_j^max of the rate axes (Section 2): homogeneous
 * Neumann as in eq (bound1), or the payoff (Dirichlet) as in eq (bound1_0).  The lower faces carry the
 * payoff and V = V^max is Neumann in both. */
enum { ORC_BC_NEUMANN = 0, ORC_BC_DIRICHLET = 1 };
/* Matrix W of the W-method (row-s): the AMF-refined W of eq (Wmat1), or the lower triangle P of the
 * semi-discrete matrix (diagonal included), which turns a fixed number of Gauss-Seidel sweeps of the
 * theta-method into a W-method (Section 4.2, eqs (thetamet) and (GS)). */
enum { ORC_W_AMF = 0, ORC_W_LOWER = 1 };

typedef struct {
    int32_t N;          /* spatial dimension: N-1 forward rates plus the volatility V            */
    int32_t model;      /* ORC_SABR_LMM or ORC_CONST_COEF                                         */
    int32_t payoff;     /* ORC_CAPLET, ORC_SWAPTION or ORC_GAUSSIAN                               */
    int32_t bc;         /* ORC_BC_NEUMANN (eq bound1) or ORC_BC_DIRICHLET (eq bound1_0)           */
    double beta, sigma; /* elasticity beta, volatility of volatility sigma                        */
    double alpha[ORC_MAXD], phi[ORC_MAXD], tau[ORC_MAXD];
    double rho[ORC_MAXD * ORC_MAXD];   /* rho[i*ORC_MAXD+j] between forward rates i, j             */
    double xmax[ORC_MAXD];             /* F_i^max ..., V^max                                       */
    double T;                          /* time to maturity (PDE horizon)                           */
    double K;                          /* strike                                                   */
    double xeval[ORC_MAXD];            /* evaluation point (F_1(0), ..., V(0))                     */
    double discount;                   /* price = discount * u(T, xeval)                           */
    double D[ORC_MAXD * ORC_MAXD];     /* CONST_COEF: symmetric diffusion matrix                   */
    double c[ORC_MAXD];                /* CONST_COEF: advection (used on axes 2..N-1, as Sketch 1) */
    double gcenter[ORC_MAXD];          /* GAUSSIAN payoff centre                                   */
    double gwidth;                     /* GAUSSIAN payoff width                                    */
} orc_problem;

/* Generic s-stage AMFR-W method, eq (row-s) with the AMF-refined W of eq (Wmat1), stage form (amfrw). */
typedef struct {
    int32_t s;
    int32_t wkind;      /* ORC_W_AMF or ORC_W_LOWER                                                */
    double a[ORC_MAXS * ORC_MAXS];  /* a[r*ORC_MAXS+j], j<r */
    double q[ORC_MAXS * ORC_MAXS];
    double b[ORC_MAXS];
    double theta, nu;
} orc_scheme;

/* Uniform grid of Section 3: M_i+1 points per axis, h_i = x_i^max / M_i, numbering theta_0. */
typedef struct {
    int N;
    long M[ORC_MAXD];
    double h[ORC_MAXD];
    long E[ORC_MAXD];   /* E_1 = 1, E_i = prod_{r<i} (M_r+1) */
    long size;          /* prod (M_i + 1) */
} orc_grid;

static void grid_make(orc_grid* G, const orc_problem* P, const int32_t* levels)
{
    G->N = P->N;
    long e = 1;
    for (int i = 0; i < P->N; ++i) {
        G->M[i] = 1L << levels[i];
        G->h[i] = P->xmax[i] / (double)G->M[i];
        G->E[i] = e;
        e *= G->M[i] + 1;
    }
    G->size = e;
}

/* Inverse of theta_0 by repeated Euclidean division (Lemma algor1 with m_i = 0). */
static void decode(const orc_grid* G, long J, long* j)
{
    long c = J;
    for (int i = 0; i < G->N; ++i) {
        j[i] = c % (G->M[i] + 1);
        c = (c - j[i]) / (G->M[i] + 1);
    }
}

/* A node is Outer (its value is boundary data, its equation Y_J' = 0) when it lies on a lower face
 * (Section 3), or, with the boundary conditions of eq (bound1_0), on the upper face of a rate axis. */
static int is_outer(const orc_problem* P, const orc_grid* G, const long* j)
{
    for (int i = 0; i < G->N; ++i) {
        if (j[i] == 0) return 1;
        if (P->bc == ORC_BC_DIRICHLET && i < G->N - 1 && j[i] == G->M[i]) return 1;
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------------- */
/* Payoff g(T, F_1, ..., F_{N-1}) (Section 2).                                                     */
double orc_payoff(const orc_problem* P, const double* x)
{
    int nr = P->N - 1;
    if (P->payoff == ORC_CAPLET) {
        double v = P->tau[0] * (x[0] - P->K);
        return v > 0.0 ? v : 0.0;
    }
    if (P->payoff == ORC_SWAPTION) {
        /* max{ sum_i tau_i (F_i - K) / ((1+tau_1 F_1)...(1+tau_i F_i)), 0 } */
        double sum = 0.0, prod = 1.0;
        for (int i = 0; i < nr; ++i) {
            prod *= 1.0 + P->tau[i] * x[i];
            sum += P->tau[i] * (x[i] - P->K) / prod;
        }
        return sum > 0.0 ? sum : 0.0;
    }
    /* Gaussian bump */
    double r2 = 0.0;
    for (int i = 0; i < P->N; ++i) {
        double d = x[i] - P->gcenter[i];
        r2 += d * d;
    }
    return exp(-0.5 * r2 / (P->gwidth * P->gwidth));
}

/* Phi_beta(x, tau) = tau x^beta / (1 + tau x), below (coef_adv). */
static double Phi_beta(double x, double tau, double beta)
{
    return tau * pow(x, beta) / (1.0 + tau * x);
}

/* PDE coefficients at a node with coordinates x (x[N-1] = V): d_i, m_ik (k>i) and a_i of eqs
 * (coef_diff), (coef_mix), (coef_adv).  d[i], m[i*N+k], a[i]; a[0] = a[N-1] = 0. */
void orc_coefficients(const orc_problem* P, const double* x, double* d, double* m, double* a)
{
    int N = P->N;
    for (int i = 0; i < N * N; ++i) m[i] = 0.0;
    for (int i = 0; i < N; ++i) a[i] = 0.0;
    if (P->model == ORC_CONST_COEF) {
        for (int i = 0; i < N; ++i) {
            d[i] = P->D[i * ORC_MAXD + i];
            for (int k = i + 1; k < N; ++k) m[i * N + k] = 2.0 * P->D[i * ORC_MAXD + k];
        }
        for (int i = 1; i < N - 1; ++i) a[i] = P->c[i];
        return;
    }
    double beta = P->beta;
    double V = x[N - 1];
    double V2 = V * V;
    /* (coef_diff) */
    for (int i = 0; i < N - 1; ++i)
        d[i] = 0.5 * P->alpha[i] * P->alpha[i] * P->rho[i * ORC_MAXD + i] * pow(x[i], 2.0 * beta) * V2;
    d[N - 1] = 0.5 * P->sigma * P->sigma * V2;
    /* (coef_mix) */
    for (int i = 0; i < N - 1; ++i) {
        for (int k = i + 1; k < N - 1; ++k)
            m[i * N + k] = P->alpha[i] * P->alpha[k] * P->rho[i * ORC_MAXD + k] * pow(x[i], beta) *
                           pow(x[k], beta) * V2;
        m[i * N + (N - 1)] = P->alpha[i] * P->sigma * P->phi[i] * pow(x[i], beta) * V2;
    }
    /* (coef_adv): a_i for paper indices i = 2..N-1, inner sum over paper j = 2..i */
    for (int i = 1; i < N - 1; ++i) {
        double s = 0.0;
        for (int j = 1; j <= i; ++j)
            s += P->alpha[i] * P->alpha[j] * P->rho[i * ORC_MAXD + j] * Phi_beta(x[j], P->tau[j], beta);
        a[i] = s * pow(x[i], beta) * V2;
    }
}

/* d_i alone at a node (coef_diff), as needed by the directional systems of Lemma lema:ls. */
static double coef_diag(const orc_problem* P, const double* x, int i)
{
    int N = P->N;
    if (P->model == ORC_CONST_COEF) return P->D[i * ORC_MAXD + i];
    double V2 = x[N - 1] * x[N - 1];
    if (i == N - 1) return 0.5 * P->sigma * P->sigma * V2;
    return 0.5 * P->alpha[i] * P->alpha[i] * P->rho[i * ORC_MAXD + i] * pow(x[i], 2.0 * P->beta) * V2;
}

/* ---------------------------------------------------------------------------------------------- */
/* Sketch 1: the semi-discrete operator F(Y) of (mmnd_0) on the full vector Y (Outer rows zero).   */
static void eval_F(const orc_problem* P, const orc_grid* G, const double* Y, double* out)
{
    int N = G->N;
    long j[ORC_MAXD];
    double x[ORC_MAXD], d[ORC_MAXD], m[ORC_MAXD * ORC_MAXD], a[ORC_MAXD];
    for (long J = 0; J < G->size; ++J) {
        decode(G, J, j);
        if (is_outer(P, G, j)) {          /* J in Outer: Y_J' = 0 */
            out[J] = 0.0;
            continue;
        }
        for (int i = 0; i < N; ++i) x[i] = (double)j[i] * G->h[i];
        orc_coefficients(P, x, d, m, a);
        double acc = 0.0;
        /* second differences, with the Neumann ghost value Y_{J+E_i} := Y_{J-E_i} at j_i = M_i */
        for (int i = 0; i < N; ++i) {
            double h2 = G->h[i] * G->h[i];
            double lap;
            if (j[i] != G->M[i])
                lap = (Y[J + G->E[i]] - 2.0 * Y[J] + Y[J - G->E[i]]) / h2;
            else
                lap = (2.0 * Y[J - G->E[i]] - 2.0 * Y[J]) / h2;
            acc += d[i] * lap;
        }
        /* mixed differences, zero when either index sits on its upper (Neumann) face */
        for (int i = 0; i < N - 1; ++i) {
            for (int k = i + 1; k < N; ++k) {
                double mix = 0.0;
                if (j[i] != G->M[i] && j[k] != G->M[k]) {
                    long Ei = G->E[i], Ek = G->E[k];
                    mix = (Y[J + Ei + Ek] + Y[J - Ei - Ek] - Y[J + Ei - Ek] - Y[J - Ei + Ek]) /
                          (4.0 * G->h[i] * G->h[k]);
                }
                acc += m[i * N + k] * mix;
            }
        }
        /* first differences (advection) for paper axes 2..N-1, zero on the upper face */
        for (int i = 1; i < N - 1; ++i) {
            double grad = 0.0;
            if (j[i] != G->M[i]) grad = (Y[J + G->E[i]] - Y[J - G->E[i]]) / (2.0 * G->h[i]);
            acc += a[i] * grad;
        }
        out[J] = acc;
    }
}

/* Textbook Thomas algorithm for sub/diag/super (lo[0] and up[n-1] unused). */
static void thomas(long n, const double* lo, const double* di, const double* up, const double* r,
                   double* x, double* cp, double* dp)
{
    cp[0] = up[0] / di[0];
    dp[0] = r[0] / di[0];
    for (long k = 1; k < n; ++k) {
        double den = di[k] - lo[k] * cp[k - 1];
        cp[k] = (k < n - 1) ? up[k] / den : 0.0;
        dp[k] = (r[k] - lo[k] * dp[k - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (long k = n - 2; k >= 0; --k) x[k] = dp[k] - cp[k] * x[k + 1];
}

/* Lemma lema:ls: (I - nu dt A_i) K = G along axis i, as prod_{k != i} M_k tridiagonal systems of
 * size M_i (decomp1) with (delta_i)_J = (d_i)_J / h_i^2.  Outer entries: K_J = G_J (= 0).  With the
 * Dirichlet faces of eq (bound1_0) a rate axis has the unknowns j_i = 1..M_i - 1 only: its systems
 * have size M_i - 1 and the neighbour on the upper face is an Outer node (K = 0 there). */
static void solve_axis(const orc_problem* P, const orc_grid* G, int ax, double nudt, const double* Gv,
                       double* K)
{
    int N = G->N;
    long Mi = G->M[ax];
    const int dir = P->bc == ORC_BC_DIRICHLET && ax < N - 1;
    long n = dir ? Mi - 1 : Mi;          /* unknowns along the line */
    size_t cap = (size_t)(Mi > 0 ? Mi : 1);
    double *lo = malloc(sizeof(double) * cap), *di = malloc(sizeof(double) * cap);
    double *up = malloc(sizeof(double) * cap), *r = malloc(sizeof(double) * cap);
    double *xs = malloc(sizeof(double) * cap), *cp = malloc(sizeof(double) * cap);
    double *dp = malloc(sizeof(double) * cap);
    long j[ORC_MAXD];
    double x[ORC_MAXD];
    double h2 = G->h[ax] * G->h[ax];
    for (long J = 0; J < G->size; ++J) K[J] = Gv[J];
    for (long J0 = 0; n > 0 && J0 < G->size; ++J0) {
        decode(G, J0, j);
        /* one system per multi-index with j_ax = 1 and every other index on an unknown */
        if (j[ax] != 1) continue;
        if (is_outer(P, G, j)) continue;
        for (long t = 1; t <= n; ++t) {
            long J = J0 + (t - 1) * G->E[ax];
            for (int i = 0; i < N; ++i) x[i] = (double)j[i] * G->h[i];
            x[ax] = (double)t * G->h[ax];
            double delta = coef_diag(P, x, ax) / h2;
            long row = t - 1;
            di[row] = 1.0 + 2.0 * nudt * delta;
            /* the Neumann ghost Y_{J+E} = Y_{J-E} doubles the sub-diagonal of the last row */
            lo[row] = (t == 1) ? 0.0 : ((t == Mi && !dir) ? -2.0 * nudt * delta : -nudt * delta);
            up[row] = (t == n) ? 0.0 : -nudt * delta;
            r[row] = Gv[J];
        }
        thomas(n, lo, di, up, r, xs, cp, dp);
        for (long t = 1; t <= n; ++t) K[J0 + (t - 1) * G->E[ax]] = xs[t - 1];
    }
    free(lo); free(di); free(up); free(r); free(xs); free(cp); free(dp);
}

/* Row J of the semi-discrete matrix A of Sketch 1 (F(Y) = A Y) for an inner node J with multi-index
 * j: appends the column indices and values of its nonzero entries (with repeats: the Neumann ghost
 * adds to J - E_i).  Up to 1 + 2N + 4 N(N-1)/2 entries. */
static int row_of_A(const orc_problem* P, const orc_grid* G, long J, const long* j, long* col,
                    double* val)
{
    int N = G->N, n = 0;
    double x[ORC_MAXD], d[ORC_MAXD], m[ORC_MAXD * ORC_MAXD], a[ORC_MAXD];
    for (int i = 0; i < N; ++i) x[i] = (double)j[i] * G->h[i];
    orc_coefficients(P, x, d, m, a);
    for (int i = 0; i < N; ++i) {
        double c = d[i] / (G->h[i] * G->h[i]);
        col[n] = J; val[n++] = -2.0 * c;
        if (j[i] != G->M[i]) {
            col[n] = J + G->E[i]; val[n++] = c;
            col[n] = J - G->E[i]; val[n++] = c;
        } else {
            col[n] = J - G->E[i]; val[n++] = 2.0 * c;
        }
    }
    for (int i = 0; i < N - 1; ++i)
        for (int k = i + 1; k < N; ++k) {
            if (j[i] == G->M[i] || j[k] == G->M[k]) continue;
            double c = m[i * N + k] / (4.0 * G->h[i] * G->h[k]);
            long Ei = G->E[i], Ek = G->E[k];
            col[n] = J + Ei + Ek; val[n++] = c;
            col[n] = J - Ei - Ek; val[n++] = c;
            col[n] = J + Ei - Ek; val[n++] = -c;
            col[n] = J - Ei + Ek; val[n++] = -c;
        }
    for (int i = 1; i < N - 1; ++i) {
        if (j[i] == G->M[i]) continue;
        double c = a[i] / (2.0 * G->h[i]);
        col[n] = J + G->E[i]; val[n++] = c;
        col[n] = J - G->E[i]; val[n++] = -c;
    }
    return n;
}

/* (I - thdt P) K = R by forward substitution in the order of theta_0 (Section 4.2, eq (GS)): P is the
 * lower triangle of A including its diagonal, so K_J only needs the already computed K_{J'}, J' < J.
 * Outer rows are identity rows (K_J = R_J, which is 0 for stage increments). */
static void solve_lower(const orc_problem* P, const orc_grid* G, double thdt, const double* R, double* K)
{
    long j[ORC_MAXD], col[1 + 2 * ORC_MAXD + 2 * ORC_MAXD * ORC_MAXD];
    double val[1 + 2 * ORC_MAXD + 2 * ORC_MAXD * ORC_MAXD];
    for (long J = 0; J < G->size; ++J) {
        decode(G, J, j);
        if (is_outer(P, G, j)) {
            K[J] = R[J];
            continue;
        }
        int n = row_of_A(P, G, J, j, col, val);
        double diag = 0.0, acc = R[J];
        for (int e = 0; e < n; ++e) {
            if (col[e] == J) diag += val[e];
            else if (col[e] < J) acc += thdt * val[e] * K[col[e]];
        }
        K[J] = acc / (1.0 - thdt * diag);
    }
}

/* Initial data (dis0): Y_J = g at every node, inner and outer. */
static void initial_data(const orc_problem* P, const orc_grid* G, double* Y)
{
    long j[ORC_MAXD];
    double x[ORC_MAXD];
    for (long J = 0; J < G->size; ++J) {
        decode(G, J, j);
        for (int i = 0; i < G->N; ++i) x[i] = (double)j[i] * G->h[i];
        Y[J] = orc_payoff(P, x);
    }
}

/* One step of the s-stage W-method (row-s).  With the AMF-refined W of eq (Wmat1) every stage is the
 * recursion of eq (amfrw):
 *   K_r^(0) = dt F(Y_n + sum_j a_rj K_j) + sum_j q_rj K_j
 *   (I - nu dt A_i) K_r^(i) = K_r^(i-1), i = 1..N
 *   Khat_r^(0) = 2 K_r^(0) - (I - theta dt F'(Y_n)) K_r^(N)      with F'(Y_n) K = F(K)  (linear F)
 *   (I - nu dt A_i) Khat_r^(i) = Khat_r^(i-1), i = 1..N
 *   K_r = Khat_r^(N);
 * with W = P (Section 4.2) the stage is (I - theta dt P) K_r = K_r^(0).  Then Y_{n+1} = Y_n + sum_r b_r K_r. */
static void amfrw_step(const orc_problem* P, const orc_grid* G, const orc_scheme* S, double dt,
                       double* Y, double** Kst, double* Z, double* K0, double* X, double* FX)
{
    long n = G->size;
    for (int r = 0; r < S->s; ++r) {
        for (long J = 0; J < n; ++J) {
            double z = Y[J];
            for (int jj = 0; jj < r; ++jj) z += S->a[r * ORC_MAXS + jj] * Kst[jj][J];
            Z[J] = z;
        }
        eval_F(P, G, Z, FX);
        for (long J = 0; J < n; ++J) {
            double k0 = dt * FX[J];
            for (int jj = 0; jj < r; ++jj) k0 += S->q[r * ORC_MAXS + jj] * Kst[jj][J];
            K0[J] = k0;
        }
        if (S->wkind == ORC_W_LOWER) {
            solve_lower(P, G, S->theta * dt, K0, Kst[r]);
            continue;
        }
        memcpy(X, K0, sizeof(double) * n);
        for (int ax = 0; ax < G->N; ++ax) {
            solve_axis(P, G, ax, S->nu * dt, X, Z);
            memcpy(X, Z, sizeof(double) * n);
        }
        eval_F(P, G, X, FX);
        for (long J = 0; J < n; ++J) X[J] = 2.0 * K0[J] - X[J] + S->theta * dt * FX[J];
        for (int ax = 0; ax < G->N; ++ax) {
            solve_axis(P, G, ax, S->nu * dt, X, Z);
            memcpy(X, Z, sizeof(double) * n);
        }
        memcpy(Kst[r], X, sizeof(double) * n);
    }
    for (long J = 0; J < n; ++J) {
        double y = Y[J];
        for (int r = 0; r < S->s; ++r) y += S->b[r] * Kst[r][J];
        Y[J] = y;
    }
}

/* Tensor-product (multi)linear interpolation of the grid function Y at x (Section 5).  The cell
 * along axis i is min(floor(x_i/h_i), M_i - 1). */
static double interpolate(const orc_grid* G, const double* Y, const double* x)
{
    int N = G->N;
    long cell[ORC_MAXD];
    double t[ORC_MAXD];
    for (int i = 0; i < N; ++i) {
        long c = (long)floor(x[i] / G->h[i]);
        if (c > G->M[i] - 1) c = G->M[i] - 1;
        if (c < 0) c = 0;
        cell[i] = c;
        t[i] = (x[i] - (double)c * G->h[i]) / G->h[i];
    }
    double val = 0.0;
    for (int corner = 0; corner < (1 << N); ++corner) {
        double w = 1.0;
        long J = 0;
        for (int i = 0; i < N; ++i) {
            int up = (corner >> i) & 1;
            w *= up ? t[i] : 1.0 - t[i];
            J += (cell[i] + up) * G->E[i];
        }
        val += w * Y[J];
    }
    return val;
}

/* ============================ exported entry points =========================================== */

int32_t orc_abi(void) { return 4; }

long orc_grid_size(int32_t N, const int32_t* levels)
{
    long s = 1;
    for (int i = 0; i < N; ++i) s *= (1L << levels[i]) + 1;
    return s;
}

/* Paper's AMFR-W2 (coef_W2): a21 = 2/3, q21 = -4/3, b = (5/4, 3/4), theta = (3+sqrt 3)/6.
 * nu is not printed; nu = theta is the reading (it reproduces the paper's few-step tables). */
void orc_scheme_amfrw2(orc_scheme* S)
{
    memset(S, 0, sizeof(*S));
    S->s = 2;
    S->a[1 * ORC_MAXS + 0] = 2.0 / 3.0;
    S->q[1 * ORC_MAXS + 0] = -4.0 / 3.0;
    S->b[0] = 5.0 / 4.0;
    S->b[1] = 3.0 / 4.0;
    S->theta = (3.0 + sqrt(3.0)) / 6.0;
    S->nu = S->theta;
}

/* theta-method with s Gauss-Seidel sweeps as a W-method (Section 4.2): W = P, a_rj = theta,
 * q_rj = -1, b_r = 1. */
void orc_scheme_theta_gs(double theta, int32_t s, orc_scheme* S)
{
    memset(S, 0, sizeof(*S));
    S->s = s;
    S->wkind = ORC_W_LOWER;
    for (int r = 0; r < s; ++r) {
        S->b[r] = 1.0;
        for (int jj = 0; jj < r; ++jj) {
            S->a[r * ORC_MAXS + jj] = theta;
            S->q[r * ORC_MAXS + jj] = -1.0;
        }
    }
    S->theta = theta;
    S->nu = theta;
}

void orc_solve_lower(const orc_problem* P, const int32_t* levels, double thdt, const double* R, double* K)
{
    orc_grid G;
    grid_make(&G, P, levels);
    solve_lower(P, &G, thdt, R, K);
}

void orc_initial_data(const orc_problem* P, const int32_t* levels, double* Y)
{
    orc_grid G;
    grid_make(&G, P, levels);
    initial_data(P, &G, Y);
}

void orc_eval_F(const orc_problem* P, const int32_t* levels, const double* Y, double* out)
{
    orc_grid G;
    grid_make(&G, P, levels);
    eval_F(P, &G, Y, out);
}

void orc_solve_axis(const orc_problem* P, const int32_t* levels, int32_t axis, double nudt,
                    const double* Gv, double* K)
{
    orc_grid G;
    grid_make(&G, P, levels);
    solve_axis(P, &G, axis, nudt, Gv, K);
}

double orc_interpolate(const orc_problem* P, const int32_t* levels, const double* Y, const double* x)
{
    orc_grid G;
    grid_make(&G, P, levels);
    return interpolate(&G, Y, x);
}

/* Advance Y (full vector, initial data already in it) by `steps` AMFR-W steps of dt = T/total_steps
 * starting at step index 0.  Returns 0, or -1 on allocation failure. */
int32_t orc_advance(const orc_problem* P, const int32_t* levels, const orc_scheme* S, double dt,
                    int32_t steps, double* Y)
{
    orc_grid G;
    grid_make(&G, P, levels);
    long n = G.size;
    double* buf = malloc(sizeof(double) * n * (size_t)(4 + S->s));
    if (!buf) return -1;
    double* Kst[ORC_MAXS];
    for (int r = 0; r < S->s; ++r) Kst[r] = buf + (size_t)(4 + r) * n;
    for (int st = 0; st < steps; ++st) amfrw_step(P, &G, S, dt, Y, Kst, buf, buf + n, buf + 2 * n, buf + 3 * n);
    free(buf);
    return 0;
}

/* Solve on one grid from t = 0 to T with `steps` uniform steps; Y receives the final full vector. */
int32_t orc_solve_grid(const orc_problem* P, const int32_t* levels, const orc_scheme* S, int32_t steps,
                       double* Y)
{
    orc_initial_data(P, levels, Y);
    return orc_advance(P, levels, S, P->T / (double)steps, steps, Y);
}

static double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

/* Component grids of the (modified) combination technique, eqs (standardCombTechnique) and
 * (modifiedCombTechnique): for q = 0..d-1 every l in N_0^d with |l|_1 = n - q, grid levels psi + l_i,
 * coefficient (-1)^q C(d-1, q).  Enumeration order: q ascending, then l in lexicographic order with
 * the last component varying fastest.  Writes up to `cap` grids; returns the total count. */
long orc_ct_grids(int32_t d, int32_t n, int32_t psi, int32_t* levels_out, double* coef_out, long cap)
{
    long count = 0;
    int l[ORC_MAXD];
    for (int q = 0; q < d; ++q) {
        int target = n - q;
        if (target < 0) continue;
        double coef = ((q & 1) ? -1.0 : 1.0) * binom(d - 1, q);
        /* odometer over l_0..l_{d-2} in [0, target]; l_{d-1} = target - sum */
        for (int i = 0; i < d; ++i) l[i] = 0;
        for (;;) {
            int s = 0;
            for (int i = 0; i < d - 1; ++i) s += l[i];
            if (s <= target) {
                l[d - 1] = target - s;
                if (count < cap) {
                    for (int i = 0; i < d; ++i) levels_out[count * d + i] = psi + l[i];
                    coef_out[count] = coef;
                }
                ++count;
            }
            int pos = d - 2;
            while (pos >= 0) {
                if (++l[pos] <= target) break;
                l[pos] = 0;
                --pos;
            }
            if (pos < 0) break;
        }
    }
    return count;
}

/* Price by the combination technique (or a full grid when n_grids == 1, coef = 1): every component
 * grid solved independently (OpenMP dynamic schedule, one grid per thread, as the paper does), its
 * solution interpolated at xeval, then sum_l c_l u_l(xeval) times the discount, in grid order.
 * unit_vals (optional) receives u_l(xeval) per grid.  Returns 0 or -1. */
int32_t orc_price_grids(const orc_problem* P, const int32_t* levels, const double* coef, int32_t n_grids,
                        const orc_scheme* S, int32_t steps, int32_t nthreads, double* unit_vals,
                        double* price)
{
    int d = P->N;
    double* vals = malloc(sizeof(double) * (size_t)n_grids);
    int fail = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
#endif
    for (int g = 0; g < n_grids; ++g) {
        const int32_t* lv = levels + (size_t)g * d;
        long sz = orc_grid_size(d, lv);
        double* Y = malloc(sizeof(double) * sz);
        if (!Y || orc_solve_grid(P, lv, S, steps, Y) != 0) {
            fail |= 1;
            vals[g] = 0.0;
        } else {
            vals[g] = orc_interpolate(P, lv, Y, P->xeval);
        }
        free(Y);
    }
    double sum = 0.0;
    for (int g = 0; g < n_grids; ++g) {
        sum += coef[g] * vals[g];
        if (unit_vals) unit_vals[g] = vals[g];
    }
    *price = P->discount * sum;
    free(vals);
    return fail ? -1 : 0;
}

int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
