/*
 * lbm_oracle.c -- plain FP64 CPU oracle of one coupled time step of the central-moment (CM)
 * pseudopotential lattice Boltzmann method with a finite-difference temperature equation
 * (Saito, De Rosis, Fei, Luo, Ebihara, Kaneko, Abe, "Lattice Boltzmann modeling and simulation of
 * forced-convection boiling on a cylinder", arXiv:1912.02018).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header or table with the HIP
 * implementation: every formula below is written out again from the paper.
 *
 * Deliberately slow and literal:
 *   * the CM transform T(u) is built numerically from the monomials of c - u (eq. matrix), and
 *     the post-collision populations are obtained by an LU solve of T(u) f* = k*;
 *   * k, k^eq and R are evaluated as T f, T f^eq and T F with f^eq from the full Hermite
 *     expansion (eq. equi) and F from the Hermite forcing term (eq. forcingTerm), and the
 *     post-collision moments follow the general relation (eq. posColl0) with the corrected
 *     force moments (eq. force2);
 *   * the pseudopotential force sums all 24 neighbours (eq. interForce), the temperature
 *     equation (eq. energy) is discretised with the same isotropic stencil, a third-order
 *     upwind convection term and classical Runge-Kutta stages.
 * Points where the paper is silent are resolved by the readings listed in the repository's
 * design notes; each is marked "reading" below.
 *
 * Storage: node (x, y) has index y*nx + x; populations are stored as f[i*nx*ny + index] in the
 * paper's velocity order.  The persistent state is the post-collision population set f* of the
 * previous step, the outlet history (post-streaming populations 2, 6, 8 of the last column from
 * the previous step) and the temperature field; one step streams, collides and advances T.
 */
#include <math.h>
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------------ */
/* Parameters (a struct of the oracle's own)                                                   */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int32_t nx, ny;
    int32_t bc_x;         /* 0: periodic in x; 1: velocity inlet at x=0, convective outlet at x=nx-1;
                             2: heated no-slip wall at x=-1/2 (T_w), convective outlet at x=nx-1 */
    int32_t rk_stages;    /* 0: isothermal, 2: Heun, 4: classical RK4 */
    int32_t warmup_steps; /* steps with neither forcing nor temperature update */
    int32_t cyl_x, cyl_y, cyl_r; /* cylinder centre and radius (lattice units); r <= 0: none */
    int32_t upwind_kind;  /* 0: third-order upwind (1/12 dissipation), 1: Kawamura-Kuwahara (1/4) */
    int32_t diag_every;   /* accumulate Nu every diag_every steps (0: never) */
    double nu;            /* kinematic viscosity; omega = (nu/cs^2 + 1/2)^-1 */
    double eos_a, eos_b, eos_R, acentric;
    double Tr_sat;        /* saturation temperature / T_c */
    double dTr_wall;      /* wall superheat / T_c */
    double G, sigma;
    double gx, gy;        /* body-force acceleration */
    double rho_gref;      /* F_g = (rho - rho_gref) g; < 0 selects rho_l */
    double rho_l, rho_v;  /* coexistence densities; <= 0 selects the Maxwell construction */
    double rho_wall;      /* density given to solid nodes; <= 0 selects rho_l */
    double u_in;          /* inlet velocity */
    double alpha_T;       /* thermal diffusivity (of the liquid when the vapour value is set) */
    double cv;            /* specific heat at constant volume */
    double nu_vapor;      /* vapour kinematic viscosity; <= 0: nu in both phases */
    double alpha_vapor;   /* vapour thermal diffusivity; <= 0: alpha_T in both phases */
    int32_t outlet_kind;  /* speed of the convective outlet: 0 u_in; 1 the local outflow velocity */
} orc_params;

/* ------------------------------------------------------------------------------------------ */
/* D2Q9 lattice (eq. velVec) and the 24-neighbour interaction stencil (eq. interForce)          */
/* ------------------------------------------------------------------------------------------ */
static const int CX[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
static const int CY[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
static const int OPP[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
static double lattice_w(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }
static const double CS2 = 1.0 / 3.0;

/* weights w(|e|^2) of the pseudo-D2Q25 stencil, 6th-order isotropic */
static double stencil_w(int e2)
{
    switch (e2) {
    case 1: return 4.0 / 21.0;
    case 2: return 4.0 / 45.0;
    case 4: return 1.0 / 60.0;
    case 5: return 2.0 / 315.0;
    case 8: return 1.0 / 5040.0;
    default: return 0.0;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Peng-Robinson equation of state (eq. eos)                                                   */
/* ------------------------------------------------------------------------------------------ */
/* T_c from the PR relations a = 0.4572 R^2 Tc^2/pc and b = 0.0778 R Tc/pc (reading: the formula,
 * not the rounded printed 0.1094) */
double orc_Tc(const orc_params *p) { return 0.0778 * p->eos_a / (0.4572 * p->eos_b * p->eos_R); }
double orc_pc(const orc_params *p) { return 0.0778 * p->eos_R * orc_Tc(p) / p->eos_b; }

static double pr_kappa(double w) { return 0.37464 + 1.54226 * w - 0.26992 * w * w; }

double orc_phi(const orc_params *p, double T)
{
    double s = 1.0 + pr_kappa(p->acentric) * (1.0 - sqrt(T / orc_Tc(p)));
    return s * s;
}

/* d(phi)/dT */
double orc_dphi_dT(const orc_params *p, double T)
{
    double Tc = orc_Tc(p), k = pr_kappa(p->acentric);
    double s = 1.0 + k * (1.0 - sqrt(T / Tc));
    /* d/dT sqrt(T/Tc) = 1/(2 sqrt(T Tc)) */
    return 2.0 * s * (-k) / (2.0 * sqrt(T * Tc));
}

double orc_eos_p(const orc_params *p, double rho, double T)
{
    double a = p->eos_a, b = p->eos_b, R = p->eos_R;
    return rho * R * T / (1.0 - b * rho) - a * orc_phi(p, T) * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}

/* (dp/dT) at constant density */
double orc_eos_dpdT(const orc_params *p, double rho, double T)
{
    double a = p->eos_a, b = p->eos_b, R = p->eos_R;
    return rho * R / (1.0 - b * rho) - a * orc_dphi_dT(p, T) * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}

/* dp/drho at constant T (used only to locate the spinodals for the Maxwell construction) */
double orc_eos_dpdrho(const orc_params *p, double rho, double T)
{
    double a = p->eos_a, b = p->eos_b, R = p->eos_R;
    double d1 = 1.0 - b * rho, d2 = 1.0 + 2.0 * b * rho - b * b * rho * rho;
    return R * T / (d1 * d1) - a * orc_phi(p, T) * (2.0 * rho * d2 - rho * rho * (2.0 * b - 2.0 * b * b * rho)) / (d2 * d2);
}

/* pseudopotential consistent with the EOS (eq. potential); NaN when the radicand is negative */
double orc_psi(const orc_params *p, double rho, double T)
{
    double rad = 2.0 * (orc_eos_p(p, rho, T) - rho * CS2) / (p->G * CS2);
    return sqrt(rad);
}

/* ------------------------------------------------------------------------------------------ */
/* Maxwell equal-area construction (reading: equal area in specific volume v = 1/rho)          */
/* ------------------------------------------------------------------------------------------ */
/* antiderivative of p(v) dv for PR: RT ln(v-b) - a phi/(2 sqrt2 b) ln((v+b-sqrt2 b)/(v+b+sqrt2 b)) */
static double pr_int_pdv(const orc_params *p, double v, double T)
{
    double a = p->eos_a, b = p->eos_b, R = p->eos_R, s2 = sqrt(2.0);
    return R * T * log(v - b) - a * orc_phi(p, T) / (2.0 * s2 * b) * log((v + b - s2 * b) / (v + b + s2 * b));
}

/* bisection for f(rho) = target on [lo, hi] where f is monotonic */
static double bisect_p(const orc_params *p, double T, double target, double lo, double hi)
{
    double flo = orc_eos_p(p, lo, T) - target;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        double fm = orc_eos_p(p, mid, T) - target;
        if ((fm > 0) == (flo > 0)) { lo = mid; flo = fm; } else { hi = mid; }
        if (hi - lo <= 1e-16 * hi) break;
    }
    return 0.5 * (lo + hi);
}

static double bisect_dpdrho(const orc_params *p, double T, double lo, double hi)
{
    double flo = orc_eos_dpdrho(p, lo, T);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        double fm = orc_eos_dpdrho(p, mid, T);
        if ((fm > 0) == (flo > 0)) { lo = mid; flo = fm; } else { hi = mid; }
        if (hi - lo <= 1e-16 * hi) break;
    }
    return 0.5 * (lo + hi);
}

/* Returns 0 on success. Below T_c the isotherm has a vapour spinodal (local max of p) and a liquid
 * spinodal (local min); for a trial pressure between them the outer roots give v_l and v_v, and
 * the trial pressure is bisected until the area between the isotherm and the line vanishes. */
int orc_maxwell(const orc_params *p, double T, double *rho_v, double *rho_l, double *p_sat)
{
    double b = p->eos_b, rmax = 1.0 / b;
    /* locate the two spinodals by scanning dp/drho */
    double sp[2];
    int nsp = 0;
    int nscan = 20000;
    double prev = orc_eos_dpdrho(p, 1e-6, T);
    for (int k = 1; k <= nscan && nsp < 2; ++k) {
        double r0 = 1e-6 + (rmax * 0.999 - 1e-6) * (k - 1) / nscan;
        double r1 = 1e-6 + (rmax * 0.999 - 1e-6) * k / nscan;
        double cur = orc_eos_dpdrho(p, r1, T);
        if ((cur > 0) != (prev > 0)) sp[nsp++] = bisect_dpdrho(p, T, r0, r1);
        prev = cur;
    }
    if (nsp < 2) return -1;
    double pmax = orc_eos_p(p, sp[0], T), pmin = orc_eos_p(p, sp[1], T);
    double lo = pmin > 0 ? pmin : 1e-14, hi = pmax;
    double rv = 0, rl = 0, ps = 0;
    for (int it = 0; it < 200; ++it) {
        ps = 0.5 * (lo + hi);
        rv = bisect_p(p, T, ps, 1e-12, sp[0]);
        rl = bisect_p(p, T, ps, sp[1], rmax * 0.999999);
        double vl = 1.0 / rl, vv = 1.0 / rv;
        /* area = int_{vl}^{vv} (p - ps) dv */
        double area = pr_int_pdv(p, vv, T) - pr_int_pdv(p, vl, T) - ps * (vv - vl);
        /* larger ps -> smaller area */
        if (area > 0) lo = ps; else hi = ps;
        if (hi - lo <= 1e-16 * hi) break;
    }
    *rho_v = rv;
    *rho_l = rl;
    *p_sat = ps;
    return 0;
}

/* latent heat from the Clausius-Clapeyron relation on the Maxwell coexistence curve (reading of
 * "determined from the EOS"): h_fg = T (1/rho_v - 1/rho_l) dp_sat/dT, central difference in T */
double orc_hfg(const orc_params *p, double T)
{
    double h = 1e-5 * T, rv, rl, ps, rv1, rl1, p1, rv2, rl2, p2;
    if (orc_maxwell(p, T, &rv, &rl, &ps) || orc_maxwell(p, T + h, &rv1, &rl1, &p1) || orc_maxwell(p, T - h, &rv2, &rl2, &p2))
        return NAN;
    return T * (1.0 / rv - 1.0 / rl) * (p1 - p2) / (2.0 * h);
}

/* ------------------------------------------------------------------------------------------ */
/* Equilibrium, forcing term and the CM transform                                               */
/* ------------------------------------------------------------------------------------------ */
/* full Hermite equilibrium up to fourth order (eq. equi) */
void orc_feq(double rho, double ux, double uy, double *feq)
{
    for (int i = 0; i < 9; ++i) {
        double cx = CX[i], cy = CY[i];
        double H2xx = cx * cx - CS2, H2yy = cy * cy - CS2, H2xy = cx * cy;
        double H3xxy = (cx * cx - CS2) * cy, H3xyy = cx * (cy * cy - CS2);
        double H4xxyy = (cx * cx - CS2) * (cy * cy - CS2);
        double t1 = (cx * ux + cy * uy) / CS2;
        double t2 = (H2xx * ux * ux + 2.0 * H2xy * ux * uy + H2yy * uy * uy) / (2.0 * CS2 * CS2);
        double t3 = (H3xxy * ux * ux * uy + H3xyy * ux * uy * uy) / (2.0 * CS2 * CS2 * CS2);
        double t4 = H4xxyy * ux * ux * uy * uy / (4.0 * CS2 * CS2 * CS2 * CS2);
        feq[i] = lattice_w(i) * rho * (1.0 + t1 + t2 + t3 + t4);
    }
}

/* Hermite forcing term (eq. forcingTerm): sum over orders n of H^(n) contracted with the
 * symmetrised products [F u ... u], divided by n! cs^(2n); only the third- and fourth-order
 * components representable on D2Q9 (xxy, xyy, xxyy) are kept. */
void orc_force_pop(double Fx, double Fy, double ux, double uy, double *Fi)
{
    for (int i = 0; i < 9; ++i) {
        double cx = CX[i], cy = CY[i];
        double H2xx = cx * cx - CS2, H2yy = cy * cy - CS2, H2xy = cx * cy;
        double H3xxy = (cx * cx - CS2) * cy, H3xyy = cx * (cy * cy - CS2);
        double H4xxyy = (cx * cx - CS2) * (cy * cy - CS2);
        /* order 1: H1 . F / cs^2 */
        double t1 = (cx * Fx + cy * Fy) / CS2;
        /* order 2: H2 : (F u + u F) / (2 cs^4) */
        double Fu_xx = 2.0 * Fx * ux, Fu_yy = 2.0 * Fy * uy, Fu_xy = Fx * uy + ux * Fy;
        double t2 = (H2xx * Fu_xx + 2.0 * H2xy * Fu_xy + H2yy * Fu_yy) / (2.0 * CS2 * CS2);
        /* order 3: each of xxy and xyy occurs in 3 index orders; [Fuu]_xxy = 2 Fx ux uy + Fy ux^2 */
        double Fuu_xxy = 2.0 * Fx * ux * uy + Fy * ux * ux;
        double Fuu_xyy = 2.0 * Fy * ux * uy + Fx * uy * uy;
        double t3 = 3.0 * (H3xxy * Fuu_xxy + H3xyy * Fuu_xyy) / (6.0 * CS2 * CS2 * CS2);
        /* order 4: xxyy occurs in 6 index orders; [Fuuu]_xxyy = 2 Fx ux uy^2 + 2 Fy ux^2 uy */
        double Fuuu_xxyy = 2.0 * Fx * ux * uy * uy + 2.0 * Fy * ux * ux * uy;
        double t4 = 6.0 * H4xxyy * Fuuu_xxyy / (24.0 * CS2 * CS2 * CS2 * CS2);
        Fi[i] = lattice_w(i) * (t1 + t2 + t3 + t4);
    }
}

/* CM transform T(u) (eq. matrix): rows are the monomials of the shifted velocities cbar = c - u */
void orc_T_matrix(double ux, double uy, double *T)
{
    for (int i = 0; i < 9; ++i) {
        double bx = CX[i] - ux, by = CY[i] - uy;
        T[0 * 9 + i] = 1.0;
        T[1 * 9 + i] = bx;
        T[2 * 9 + i] = by;
        T[3 * 9 + i] = bx * bx + by * by;
        T[4 * 9 + i] = bx * bx - by * by;
        T[5 * 9 + i] = bx * by;
        T[6 * 9 + i] = bx * bx * by;
        T[7 * 9 + i] = bx * by * by;
        T[8 * 9 + i] = bx * bx * by * by;
    }
}

static void matvec9(const double *A, const double *x, double *y)
{
    for (int r = 0; r < 9; ++r) {
        double s = 0.0;
        for (int c = 0; c < 9; ++c) s += A[r * 9 + c] * x[c];
        y[r] = s;
    }
}

/* solve A x = b by Gaussian elimination with partial pivoting (A, b are overwritten) */
int orc_lu_solve9(double *A, double *b, double *x)
{
    int n = 9;
    for (int k = 0; k < n; ++k) {
        int piv = k;
        double best = fabs(A[k * n + k]);
        for (int r = k + 1; r < n; ++r)
            if (fabs(A[r * n + k]) > best) { best = fabs(A[r * n + k]); piv = r; }
        if (best == 0.0) return -1;
        if (piv != k) {
            for (int c = 0; c < n; ++c) { double t = A[k * n + c]; A[k * n + c] = A[piv * n + c]; A[piv * n + c] = t; }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int r = k + 1; r < n; ++r) {
            double m = A[r * n + k] / A[k * n + k];
            for (int c = k; c < n; ++c) A[r * n + c] -= m * A[k * n + c];
            b[r] -= m * b[k];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < n; ++c) s -= A[r * n + c] * x[c];
        x[r] = s / A[r * n + r];
    }
    return 0;
}

/* Collision of one node (eq. posColl0 with the corrected force moments of eq. force2):
 *   k* = (I - K) T f + K T f^eq + (I - K/2) R',  R' = T F(u) with R'_3 = 4 a |Fm|^2,
 *   R'_8 = (4/3) a |Fm|^2, a = sigma/psi^2, K = diag[1,1,1,1,w,w,1,1,1];  then T f* = k*.
 * u is the velocity of the node (already including F/2), F the total force, Fm the
 * interaction force and psi the node's pseudopotential (Fm2_over_psi2 = |Fm|^2/psi^2). */
void orc_collide_node(double omega, double sigma, const double *f, double rho, double ux, double uy,
                      double Fx, double Fy, double Fm2_over_psi2, double *fstar)
{
    double T[81], A[81], feq[9], Fi[9], k[9], keq[9], R[9], ks[9];
    orc_T_matrix(ux, uy, T);
    orc_feq(rho, ux, uy, feq);
    orc_force_pop(Fx, Fy, ux, uy, Fi);
    matvec9(T, f, k);
    matvec9(T, feq, keq);
    matvec9(T, Fi, R);
    R[3] = 4.0 * sigma * Fm2_over_psi2;
    R[8] = (4.0 / 3.0) * sigma * Fm2_over_psi2;
    for (int m = 0; m < 9; ++m) {
        double K = (m == 4 || m == 5) ? omega : 1.0;
        ks[m] = (1.0 - K) * k[m] + K * keq[m] + (1.0 - 0.5 * K) * R[m];
    }
    memcpy(A, T, sizeof(A));
    orc_lu_solve9(A, ks, fstar);
}

/* ------------------------------------------------------------------------------------------ */
/* Simulation state                                                                            */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    orc_params p;
    int nx, ny, n;
    double Tc, T_sat, T_w, rho_l, rho_v, rho_w, rho_gref, omega;
    long step;
    unsigned char *solid; /* [n] */
    double *fstar;        /* [9][n] post-collision populations of the previous step */
    double *hist;         /* [3][ny] previous post-streaming populations 2, 6, 8 at x = nx-1 */
    double *T;            /* [n] temperature */
    /* work arrays */
    double *f, *rho, *ux, *uy, *jx, *jy, *psi, *Fx, *Fy, *Fm2p, *gradrx, *gradry, *divu;
    double *Y, *K, *acc, *Tn;
    double nu_sum;
    long nu_count;
    int unstable;
    /* probes */
    int np;
    double *probe_x, *probe_y;
} orc_sim;

static int wrapi(int a, int n) { a %= n; return a < 0 ? a + n : a; }

/* solid test, exact in integers (reading) */
static int is_solid_xy(const orc_sim *s, int x, int y)
{
    if (s->p.cyl_r <= 0) return 0;
    long dx = x - s->p.cyl_x, dy = y - s->p.cyl_y;
    return dx * dx + dy * dy <= (long)s->p.cyl_r * s->p.cyl_r;
}

int orc_is_solid(const orc_sim *s, int x, int y) { return is_solid_xy(s, x, y); }

/* ------------------------------------------------------------------------------------------ */
/* Phase-dependent transport properties (reading of the steam-table property ratios): nu and   */
/* alpha vary linearly in density between the vapour and liquid coexistence densities, held   */
/* constant outside; nu = p->nu and alpha = p->alpha_T are the liquid values.                  */
/* ------------------------------------------------------------------------------------------ */
static double phase_frac(const orc_sim *s, double rho, int *inside)
{
    double t = (rho - s->rho_v) / (s->rho_l - s->rho_v);
    *inside = t > 0.0 && t < 1.0;
    return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
}

static double nu_at(const orc_sim *s, double rho)
{
    if (s->p.nu_vapor <= 0.0) return s->p.nu;
    int in;
    double t = phase_frac(s, rho, &in);
    return s->p.nu_vapor + t * (s->p.nu - s->p.nu_vapor);
}

static double alpha_at(const orc_sim *s, double rho)
{
    if (s->p.alpha_vapor <= 0.0) return s->p.alpha_T;
    int in;
    double t = phase_frac(s, rho, &in);
    return s->p.alpha_vapor + t * (s->p.alpha_T - s->p.alpha_vapor);
}

static double dalpha_drho(const orc_sim *s, double rho)
{
    if (s->p.alpha_vapor <= 0.0) return 0.0;
    int in;
    phase_frac(s, rho, &in);
    return in ? (s->p.alpha_T - s->p.alpha_vapor) / (s->rho_l - s->rho_v) : 0.0;
}

/* ------------------------------------------------------------------------------------------ */
/* Field extension (reading): solid nodes carry rho_w, u = 0, T_w (stored directly in the      */
/* arrays); y is periodic; x is periodic, or ghost columns x < 0 copy rho and u of column 0    */
/* with T = T_sat (inlet), or behind a wall (bc 2) carry rho_w, u = 0, T_w like solid nodes,   */
/* and x >= nx copy column nx-1 (outlet).                                                      */
/* ------------------------------------------------------------------------------------------ */
enum { EXT_NODE = 0, EXT_INLET = 1, EXT_WALL = 2 };

static int ext_index(const orc_sim *s, int x, int y, int *kind)
{
    int yy = wrapi(y, s->ny), xx;
    *kind = EXT_NODE;
    if (s->p.bc_x == 0) {
        xx = wrapi(x, s->nx);
    } else if (x < 0) {
        xx = 0;
        *kind = s->p.bc_x == 2 ? EXT_WALL : EXT_INLET;
    } else if (x >= s->nx) {
        xx = s->nx - 1;
    } else {
        xx = x;
    }
    return yy * s->nx + xx;
}

/* rho (wall_value = rho_w) or a velocity component (wall_value = 0) on the extended field */
static double ext_scalar(const orc_sim *s, const double *a, int x, int y, double wall_value)
{
    int g;
    int k = ext_index(s, x, y, &g);
    return g == EXT_WALL ? wall_value : a[k];
}

static double ext_temperature(const orc_sim *s, const double *a, int x, int y)
{
    int g;
    int k = ext_index(s, x, y, &g);
    return g == EXT_INLET ? s->T_sat : (g == EXT_WALL ? s->T_w : a[k]);
}

/* ------------------------------------------------------------------------------------------ */
/* Creation and initial state                                                                  */
/* ------------------------------------------------------------------------------------------ */
static double *alloc_d(size_t n) { return (double *)calloc(n, sizeof(double)); }

static void build_probes(orc_sim *s)
{
    s->np = 0;
    if (s->p.cyl_r <= 0) return;
    double R = s->p.cyl_r;
    int np = 8 * (int)ceil(M_PI * R / 4.0);
    s->np = np;
    s->probe_x = alloc_d(np);
    s->probe_y = alloc_d(np);
    double r = R + 1.5;
    for (int k = 0; k < np; ++k) {
        double th = 2.0 * M_PI * (k + 0.5) / np;
        s->probe_x[k] = s->p.cyl_x + r * cos(th);
        s->probe_y[k] = s->p.cyl_y + r * sin(th);
    }
}

int orc_set_fields(orc_sim *s, const double *rho, const double *ux, const double *uy, const double *T);

orc_sim *orc_create(const orc_params *p)
{
    if (p->nx < 4 || p->ny < 4) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->p = *p;
    s->nx = p->nx;
    s->ny = p->ny;
    s->n = p->nx * p->ny;
    s->Tc = orc_Tc(p);
    s->T_sat = p->Tr_sat * s->Tc;
    s->T_w = s->T_sat + p->dTr_wall * s->Tc;
    s->rho_l = p->rho_l;
    s->rho_v = p->rho_v;
    if (p->rho_l <= 0.0 || p->rho_v <= 0.0) {
        double rv, rl, ps;
        if (orc_maxwell(p, s->T_sat, &rv, &rl, &ps) != 0) { free(s); return NULL; }
        s->rho_l = rl;
        s->rho_v = rv;
    }
    s->rho_w = p->rho_wall > 0.0 ? p->rho_wall : s->rho_l;
    s->rho_gref = p->rho_gref >= 0.0 ? p->rho_gref : s->rho_l;
    s->omega = 1.0 / (p->nu / CS2 + 0.5);
    size_t n = (size_t)s->n;
    s->solid = (unsigned char *)calloc(n, 1);
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) s->solid[y * s->nx + x] = (unsigned char)is_solid_xy(s, x, y);
    s->fstar = alloc_d(9 * n);
    s->f = alloc_d(9 * n);
    s->hist = alloc_d(3 * (size_t)s->ny);
    s->T = alloc_d(n);
    s->rho = alloc_d(n); s->ux = alloc_d(n); s->uy = alloc_d(n);
    s->jx = alloc_d(n); s->jy = alloc_d(n); s->psi = alloc_d(n);
    s->Fx = alloc_d(n); s->Fy = alloc_d(n); s->Fm2p = alloc_d(n);
    s->gradrx = alloc_d(n); s->gradry = alloc_d(n); s->divu = alloc_d(n);
    s->Y = alloc_d(n); s->K = alloc_d(n); s->acc = alloc_d(n); s->Tn = alloc_d(n);
    build_probes(s);
    /* default initial state (reading of the garbled initial-condition sentence): saturated
     * liquid at T_sat moving with the inlet velocity; solid nodes at T_w */
    double *r0 = alloc_d(n), *u0 = alloc_d(n), *v0 = alloc_d(n), *t0 = alloc_d(n);
    for (size_t k = 0; k < n; ++k) { r0[k] = s->rho_l; u0[k] = p->bc_x == 1 ? p->u_in : 0.0; v0[k] = 0.0; t0[k] = s->T_sat; }
    orc_set_fields(s, r0, u0, v0, t0);
    free(r0); free(u0); free(v0); free(t0);
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->solid); free(s->fstar); free(s->f); free(s->hist); free(s->T);
    free(s->rho); free(s->ux); free(s->uy); free(s->jx); free(s->jy); free(s->psi);
    free(s->Fx); free(s->Fy); free(s->Fm2p); free(s->gradrx); free(s->gradry); free(s->divu);
    free(s->Y); free(s->K); free(s->acc); free(s->Tn);
    free(s->probe_x); free(s->probe_y);
    free(s);
}

/* Set the state from macroscopic fields: the post-collision populations of the (virtual)
 * previous step are f^eq(rho, u) at every node, the outlet history is f^eq of the last column,
 * T is copied and held at T_w on solid nodes; the step counter and Nu accumulators reset. */
int orc_set_fields(orc_sim *s, const double *rho, const double *ux, const double *uy, const double *T)
{
    int nx = s->nx, ny = s->ny, n = s->n;
    for (int k = 0; k < n; ++k) {
        double feq[9];
        orc_feq(rho[k], ux[k], uy[k], feq);
        for (int i = 0; i < 9; ++i) s->fstar[(size_t)i * n + k] = feq[i];
        s->T[k] = s->solid[k] ? s->T_w : T[k];
    }
    for (int y = 0; y < ny; ++y) {
        int k = y * nx + nx - 1;
        double feq[9];
        orc_feq(rho[k], ux[k], uy[k], feq);
        s->hist[0 * ny + y] = feq[2];
        s->hist[1 * ny + y] = feq[6];
        s->hist[2 * ny + y] = feq[8];
    }
    s->step = 0;
    s->nu_sum = 0.0;
    s->nu_count = 0;
    s->unstable = 0;
    return 0;
}

/* Replace the raw state (post-collision populations, outlet history, temperature, step). */
int orc_set_state(orc_sim *s, const double *fstar, const double *hist, const double *T, long step)
{
    memcpy(s->fstar, fstar, sizeof(double) * 9 * (size_t)s->n);
    memcpy(s->hist, hist, sizeof(double) * 3 * (size_t)s->ny);
    for (int k = 0; k < s->n; ++k) s->T[k] = s->solid[k] ? s->T_w : T[k];
    s->step = step;
    return 0;
}

int orc_get_state(const orc_sim *s, double *fstar, double *hist, double *T, long *step)
{
    if (fstar) memcpy(fstar, s->fstar, sizeof(double) * 9 * (size_t)s->n);
    if (hist) memcpy(hist, s->hist, sizeof(double) * 3 * (size_t)s->ny);
    if (T) memcpy(T, s->T, sizeof(double) * (size_t)s->n);
    if (step) *step = s->step;
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Streaming with boundary conditions (eq. streaming)                                           */
/* ------------------------------------------------------------------------------------------ */
/* Fraction q in (0,1] of the link from fluid node (x,y) towards (x,y) - c_i at which the
 * circle is crossed: the smaller root of |d - q c|^2 = R^2, d = (x,y) - centre. */
double orc_link_q(const orc_sim *s, int x, int y, int i)
{
    double dx = x - s->p.cyl_x, dy = y - s->p.cyl_y, cx = CX[i], cy = CY[i];
    double c2 = cx * cx + cy * cy, dc = dx * cx + dy * cy;
    double R = s->p.cyl_r;
    double disc = dc * dc - c2 * (dx * dx + dy * dy - R * R);
    return (dc - sqrt(disc)) / c2;
}

static int is_fluid_in_domain(const orc_sim *s, int x, int y)
{
    if (s->p.bc_x == 0) x = wrapi(x, s->nx);
    else if (x < 0 || x >= s->nx) return 0;
    y = wrapi(y, s->ny);
    return !s->solid[y * s->nx + x];
}

static double fstar_at(const orc_sim *s, int i, int x, int y)
{
    if (s->p.bc_x == 0) x = wrapi(x, s->nx);
    y = wrapi(y, s->ny);
    return s->fstar[(size_t)i * s->n + y * s->nx + x];
}

/* Post-streaming value of population i at fluid node (x,y) for every population whose source
 * node lies inside the domain; sources outside (inlet/outlet) are handled by the callers. */
static double pull_interior(const orc_sim *s, int i, int x, int y)
{
    int xs = x - CX[i], ys = y - CY[i];
    if (is_fluid_in_domain(s, xs, ys)) return fstar_at(s, i, xs, ys);
    /* the source is solid: linear interpolated bounce-back (reading of the Bouzidi variant) */
    int o = OPP[i];
    double q = orc_link_q(s, x, y, i);
    if (q < 0.5) {
        if (is_fluid_in_domain(s, x + CX[i], y + CY[i]))
            return 2.0 * q * fstar_at(s, o, x, y) + (1.0 - 2.0 * q) * fstar_at(s, o, x + CX[i], y + CY[i]);
        return fstar_at(s, o, x, y);
    }
    return fstar_at(s, o, x, y) / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * fstar_at(s, i, x, y);
}

/* Zou-He velocity inlet (reading): prescribed (u_in, 0), unknowns 1, 5, 7 at x = 0 */
void orc_zou_he(double u_in, double *f)
{
    double rho = (f[0] + f[3] + f[4] + 2.0 * (f[2] + f[6] + f[8])) / (1.0 - u_in);
    f[1] = f[2] + (2.0 / 3.0) * rho * u_in;
    f[5] = f[6] - 0.5 * (f[3] - f[4]) + rho * u_in / 6.0;
    f[7] = f[8] + 0.5 * (f[3] - f[4]) + rho * u_in / 6.0;
}

/* convective outflow, implicit upwind discretisation of df/dt + U df/dx = 0 at the last column:
 * f^{n+1}(N) = (f^n(N) + U f^{n+1}(N-1)) / (1 + U) */
double orc_convective(double U, double f_old_last, double f_new_prev)
{
    return (f_old_last + U * f_new_prev) / (1.0 + U);
}

/* Convection speed U of the outlet in row y (reading of the convective condition, whose speed the
 * paper leaves open): the inlet velocity, or the local outflow velocity -- the x velocity of the
 * outlet node's post-collision populations of the previous step, u = sum f*_i c_ix / sum f*_i,
 * taken as 0 where the fluid flows back in (a negative speed would make the upwind update unstable). */
static double outlet_speed(const orc_sim *s, int y)
{
    if (s->p.outlet_kind != 1) return s->p.u_in;
    int k = y * s->nx + s->nx - 1;
    double m = 0.0, jx = 0.0;
    for (int i = 0; i < 9; ++i) {
        double fi = s->fstar[(size_t)i * s->n + k];
        m += fi;
        jx += fi * CX[i];
    }
    double u = jx / m;
    return u > 0.0 ? u : 0.0;
}

/* fill s->f (post-streaming populations) for every fluid node; returns the new outlet history */
static void stream_all(orc_sim *s, double *new_hist)
{
    int nx = s->nx, ny = s->ny, n = s->n;
    static const int OUT_DIRS[3] = {2, 6, 8};
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            int k = y * nx + x;
            double f[9];
            if (s->solid[k]) {
                for (int i = 0; i < 9; ++i) s->f[(size_t)i * n + k] = 0.0;
                continue;
            }
            for (int i = 0; i < 9; ++i) {
                int xs = x - CX[i];
                if (s->p.bc_x != 0 && (xs < 0 || xs >= nx)) { f[i] = 0.0; continue; }
                f[i] = pull_interior(s, i, x, y);
            }
            if (s->p.bc_x != 0 && x == nx - 1) {
                double U = outlet_speed(s, y);
                for (int m = 0; m < 3; ++m) {
                    int i = OUT_DIRS[m];
                    double prev_col = pull_interior(s, i, nx - 2, y);
                    f[i] = orc_convective(U, s->hist[m * ny + y], prev_col);
                }
            }
            if (s->p.bc_x == 1 && x == 0) orc_zou_he(s->p.u_in, f);
            /* halfway bounce-back on the wall at x = -1/2: what left towards it returns reversed */
            if (s->p.bc_x == 2 && x == 0)
                for (int i = 1; i < 9; ++i)
                    if (CX[i] > 0) f[i] = fstar_at(s, OPP[i], 0, y);
            for (int i = 0; i < 9; ++i) s->f[(size_t)i * n + k] = f[i];
        }
    }
    if (s->p.bc_x != 0) {
        for (int y = 0; y < ny; ++y) {
            int k = y * nx + nx - 1;
            new_hist[0 * ny + y] = s->f[(size_t)2 * n + k];
            new_hist[1 * ny + y] = s->f[(size_t)6 * n + k];
            new_hist[2 * ny + y] = s->f[(size_t)8 * n + k];
        }
    } else {
        memcpy(new_hist, s->hist, sizeof(double) * 3 * (size_t)ny);
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Macroscopic fields, pseudopotential force, velocity                                         */
/* ------------------------------------------------------------------------------------------ */
static int forcing_on(const orc_sim *s) { return s->step >= s->p.warmup_steps; }

/* from s->f: rho, j at fluid nodes; wall values at solid nodes; psi; F; u (S1-S4) */
static void macroscopic(orc_sim *s)
{
    int nx = s->nx, ny = s->ny, n = s->n;
    const orc_params *p = &s->p;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        if (s->solid[k]) {
            s->rho[k] = s->rho_w; s->jx[k] = 0.0; s->jy[k] = 0.0;
            continue;
        }
        double r = 0, jx = 0, jy = 0;
        for (int i = 0; i < 9; ++i) {
            double fi = s->f[(size_t)i * n + k];
            r += fi;
            jx += fi * CX[i];
            jy += fi * CY[i];
        }
        s->rho[k] = r; s->jx[k] = jx; s->jy[k] = jy;
    }
    int fon = forcing_on(s);
    if (fon) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < n; ++k) s->psi[k] = orc_psi(p, s->rho[k], s->T[k]);
    }
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            int k = y * nx + x;
            double Fmx = 0, Fmy = 0, Fm2p = 0;
            if (s->solid[k]) { s->Fx[k] = 0; s->Fy[k] = 0; s->Fm2p[k] = 0; s->ux[k] = 0; s->uy[k] = 0; continue; }
            if (fon) {
                double sx = 0, sy = 0;
                for (int ey = -2; ey <= 2; ++ey)
                    for (int ex = -2; ex <= 2; ++ex) {
                        if (ex == 0 && ey == 0) continue;
                        int g;
                        int kk = ext_index(s, x + ex, y + ey, &g);
                        double ps = g == EXT_INLET ? orc_psi(p, s->rho[kk], s->T_sat)
                                  : (g == EXT_WALL ? orc_psi(p, s->rho_w, s->T_w) : s->psi[kk]);
                        double w = stencil_w(ex * ex + ey * ey);
                        sx += w * ps * ex;
                        sy += w * ps * ey;
                    }
                Fmx = -p->G * CS2 * s->psi[k] * sx;
                Fmy = -p->G * CS2 * s->psi[k] * sy;
                Fm2p = (Fmx * Fmx + Fmy * Fmy) / (s->psi[k] * s->psi[k]);
            }
            double Fx = Fmx, Fy = Fmy;
            if (fon) {
                Fx += (s->rho[k] - s->rho_gref) * p->gx;
                Fy += (s->rho[k] - s->rho_gref) * p->gy;
            }
            s->Fx[k] = Fx; s->Fy[k] = Fy; s->Fm2p[k] = Fm2p;
            s->ux[k] = (s->jx[k] + 0.5 * Fx) / s->rho[k];
            s->uy[k] = (s->jy[k] + 0.5 * Fy) / s->rho[k];
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Temperature equation (eq. energy)                                                           */
/* ------------------------------------------------------------------------------------------ */
/* frozen per-step quantities: isotropic gradient of rho and divergence of u */
static void thermal_frozen(orc_sim *s)
{
    int nx = s->nx, ny = s->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int k = y * nx + x;
            double gx = 0, gy = 0, dv = 0;
            for (int ey = -2; ey <= 2; ++ey)
                for (int ex = -2; ex <= 2; ++ex) {
                    if (ex == 0 && ey == 0) continue;
                    double w = stencil_w(ex * ex + ey * ey);
                    gx += w * ext_scalar(s, s->rho, x + ex, y + ey, s->rho_w) * ex;
                    gy += w * ext_scalar(s, s->rho, x + ex, y + ey, s->rho_w) * ey;
                    dv += w * (ext_scalar(s, s->ux, x + ex, y + ey, 0.0) * ex + ext_scalar(s, s->uy, x + ex, y + ey, 0.0) * ey);
                }
            s->gradrx[k] = gx; s->gradry[k] = gy; s->divu[k] = dv;
        }
}

/* L(Y) at every fluid node; zero at solid nodes */
static void thermal_rhs(orc_sim *s, const double *Y, double *L)
{
    int nx = s->nx, ny = s->ny;
    const orc_params *p = &s->p;
    double cd = p->upwind_kind == 1 ? 0.25 : 1.0 / 12.0;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int k = y * nx + x;
            if (s->solid[k]) { L[k] = 0.0; continue; }
            double u = s->ux[k], v = s->uy[k], r = s->rho[k], y0 = Y[k];
            /* upwind-biased convection u dY/dx + v dY/dy */
            double xm2 = ext_temperature(s, Y, x - 2, y), xm1 = ext_temperature(s, Y, x - 1, y);
            double xp1 = ext_temperature(s, Y, x + 1, y), xp2 = ext_temperature(s, Y, x + 2, y);
            double ym2 = ext_temperature(s, Y, x, y - 2), ym1 = ext_temperature(s, Y, x, y - 1);
            double yp1 = ext_temperature(s, Y, x, y + 1), yp2 = ext_temperature(s, Y, x, y + 2);
            double conv = u * (-xp2 + 8.0 * xp1 - 8.0 * xm1 + xm2) / 12.0 + fabs(u) * cd * (xp2 - 4.0 * xp1 + 6.0 * y0 - 4.0 * xm1 + xm2)
                        + v * (-yp2 + 8.0 * yp1 - 8.0 * ym1 + ym2) / 12.0 + fabs(v) * cd * (yp2 - 4.0 * yp1 + 6.0 * y0 - 4.0 * ym1 + ym2);
            /* isotropic gradient and Laplacian on the interaction stencil */
            double gx = 0, gy = 0, lap = 0;
            for (int ey = -2; ey <= 2; ++ey)
                for (int ex = -2; ex <= 2; ++ex) {
                    if (ex == 0 && ey == 0) continue;
                    double w = stencil_w(ex * ex + ey * ey);
                    double yn = ext_temperature(s, Y, x + ex, y + ey);
                    gx += w * yn * ex;
                    gy += w * yn * ey;
                    lap += 2.0 * w * (yn - y0);
                }
            /* (1/(rho cv)) div(lambda grad T) with lambda = rho cv alpha (reading) */
            /* with lambda = rho cv alpha(rho): (1/(rho cv)) div(lambda grad T)
             *   = alpha (lap T + grad rho . grad T / rho) + alpha'(rho) grad rho . grad T */
            double gg = s->gradrx[k] * gx + s->gradry[k] * gy;
            double diff = alpha_at(s, r) * (lap + gg / r) + dalpha_drho(s, r) * gg;
            /* pressure-work (latent heat) source */
            double src = -y0 / (r * p->cv) * orc_eos_dpdT(p, r, y0) * s->divu[k];
            L[k] = -conv + diff + src;
        }
}

static void thermal_update(orc_sim *s)
{
    int n = s->n;
    int st = s->p.rk_stages;
    thermal_frozen(s);
    if (st == 2) {
        /* Heun: T1 = T + L(T); T' = T + (L(T) + L(T1))/2 */
        thermal_rhs(s, s->T, s->K);
        for (int k = 0; k < n; ++k) { s->acc[k] = s->K[k]; s->Y[k] = s->T[k] + s->K[k]; }
        thermal_rhs(s, s->Y, s->K);
        for (int k = 0; k < n; ++k) s->Tn[k] = s->T[k] + 0.5 * (s->acc[k] + s->K[k]);
    } else if (st == 4) {
        /* classical RK4 */
        thermal_rhs(s, s->T, s->K);
        for (int k = 0; k < n; ++k) { s->acc[k] = s->K[k]; s->Y[k] = s->T[k] + 0.5 * s->K[k]; }
        thermal_rhs(s, s->Y, s->K);
        for (int k = 0; k < n; ++k) { s->acc[k] += 2.0 * s->K[k]; s->Y[k] = s->T[k] + 0.5 * s->K[k]; }
        thermal_rhs(s, s->Y, s->K);
        for (int k = 0; k < n; ++k) { s->acc[k] += 2.0 * s->K[k]; s->Y[k] = s->T[k] + s->K[k]; }
        thermal_rhs(s, s->Y, s->K);
        for (int k = 0; k < n; ++k) s->Tn[k] = s->T[k] + (s->acc[k] + s->K[k]) / 6.0;
    } else {
        return;
    }
    for (int k = 0; k < n; ++k) s->T[k] = s->solid[k] ? s->T_w : s->Tn[k];
}

/* ------------------------------------------------------------------------------------------ */
/* Diagnostics: mass and wall heat flux                                                        */
/* ------------------------------------------------------------------------------------------ */
static double bilinear(const orc_sim *s, const double *a, double px, double py)
{
    int x0 = (int)floor(px), y0 = (int)floor(py);
    double fx = px - x0, fy = py - y0;
    double a00 = a[y0 * s->nx + x0], a10 = a[y0 * s->nx + x0 + 1];
    double a01 = a[(y0 + 1) * s->nx + x0], a11 = a[(y0 + 1) * s->nx + x0 + 1];
    return (1 - fx) * (1 - fy) * a00 + fx * (1 - fy) * a10 + (1 - fx) * fy * a01 + fx * fy * a11;
}

/* from current s->rho (fluid nodes) and s->T: q_mean and Nu (probe estimator, reading) */
static void heat_flux_from_fields(const orc_sim *s, double *q_mean, double *nu)
{
    const orc_params *p = &s->p;
    if (s->np == 0) { *q_mean = 0.0; *nu = 0.0; return; }
    double qs = 0.0;
    for (int k = 0; k < s->np; ++k) {
        double rp = bilinear(s, s->rho, s->probe_x[k], s->probe_y[k]);
        double tp = bilinear(s, s->T, s->probe_x[k], s->probe_y[k]);
        qs += rp * p->cv * alpha_at(s, rp) * (s->T_w - tp) / 1.5;
    }
    double q = qs / s->np;
    double dT = s->T_w - s->T_sat;
    *q_mean = q;
    *nu = dT != 0.0 ? q * 2.0 * p->cyl_r / (s->rho_v * p->cv * alpha_at(s, s->rho_v) * dT) : 0.0;
}

/* evaluate macroscopic fields of the current state (streams into the work arrays) */
static void current_fields(orc_sim *s)
{
    double *tmp = alloc_d(3 * (size_t)s->ny);
    stream_all(s, tmp);
    macroscopic(s);
    free(tmp);
}

/* ------------------------------------------------------------------------------------------ */
/* One coupled step                                                                            */
/* ------------------------------------------------------------------------------------------ */
static void one_step(orc_sim *s)
{
    int n = s->n;
    double *new_hist = alloc_d(3 * (size_t)s->ny);
    stream_all(s, new_hist);                 /* streaming + boundary conditions */
    macroscopic(s);                          /* rho, j, psi, F, u */
    if (s->p.diag_every > 0 && s->step % s->p.diag_every == 0 && forcing_on(s)) {
        double q, nu;
        heat_flux_from_fields(s, &q, &nu);
        s->nu_sum += nu;
        s->nu_count += 1;
    }
    int fon = forcing_on(s);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        if (s->solid[k]) continue;
        double f[9], fs[9];
        for (int i = 0; i < 9; ++i) f[i] = s->f[(size_t)i * n + k];
        double om = s->p.nu_vapor > 0.0 ? 1.0 / (nu_at(s, s->rho[k]) / CS2 + 0.5) : s->omega;
        orc_collide_node(om, fon ? s->p.sigma : 0.0, f, s->rho[k], s->ux[k], s->uy[k], s->Fx[k], s->Fy[k], s->Fm2p[k], fs);
        for (int i = 0; i < 9; ++i) s->fstar[(size_t)i * n + k] = fs[i];
    }
    if (fon && s->p.rk_stages > 0) thermal_update(s);
    memcpy(s->hist, new_hist, sizeof(double) * 3 * (size_t)s->ny);
    free(new_hist);
    for (int k = 0; k < n; ++k)
        if (!s->solid[k] && !(s->rho[k] == s->rho[k])) s->unstable = 1;
    s->step += 1;
}

int orc_step(orc_sim *s, int nsteps)
{
    for (int t = 0; t < nsteps; ++t) one_step(s);
    return s->unstable ? -4 : 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Read-out                                                                                    */
/* ------------------------------------------------------------------------------------------ */
/* rho, u = (j + F/2)/rho, T of the current state; solid nodes report rho = 0, u = 0, T = T_w */
int orc_fields(orc_sim *s, double *rho, double *ux, double *uy, double *T, unsigned char *mask)
{
    current_fields(s);
    for (int k = 0; k < s->n; ++k) {
        int sd = s->solid[k];
        if (rho) rho[k] = sd ? 0.0 : s->rho[k];
        if (ux) ux[k] = sd ? 0.0 : s->ux[k];
        if (uy) uy[k] = sd ? 0.0 : s->uy[k];
        if (T) T[k] = s->T[k];
        if (mask) mask[k] = (unsigned char)sd;
    }
    return 0;
}

/* post-streaming populations of the current state (fluid nodes; zero at solid nodes) */
int orc_populations(orc_sim *s, double *f)
{
    current_fields(s);
    memcpy(f, s->f, sizeof(double) * 9 * (size_t)s->n);
    return 0;
}

/* force, pseudopotential and |Fm|^2/psi^2 of the current state */
int orc_forces(orc_sim *s, double *Fx, double *Fy, double *psi)
{
    current_fields(s);
    for (int k = 0; k < s->n; ++k) {
        if (Fx) Fx[k] = s->Fx[k];
        if (Fy) Fy[k] = s->Fy[k];
        if (psi) psi[k] = s->psi[k];
    }
    return 0;
}

double orc_total_mass(orc_sim *s)
{
    current_fields(s);
    double m = 0.0;
    for (int k = 0; k < s->n; ++k)
        if (!s->solid[k]) m += s->rho[k];
    return m;
}

int orc_wall_heat_flux(orc_sim *s, double *q_mean, double *nu, double *nu_time_avg)
{
    current_fields(s);
    heat_flux_from_fields(s, q_mean, nu);
    if (nu_time_avg) *nu_time_avg = s->nu_count ? s->nu_sum / s->nu_count : 0.0;
    return 0;
}

/* derived constants of the run: Tc, T_sat, T_w, rho_l, rho_v, rho_w, rho_gref, omega */
void orc_derived(const orc_sim *s, double *out8)
{
    out8[0] = s->Tc; out8[1] = s->T_sat; out8[2] = s->T_w; out8[3] = s->rho_l;
    out8[4] = s->rho_v; out8[5] = s->rho_w; out8[6] = s->rho_gref; out8[7] = s->omega;
}

int orc_probes(const orc_sim *s, double *px, double *py)
{
    for (int k = 0; k < s->np; ++k) { if (px) px[k] = s->probe_x[k]; if (py) py[k] = s->probe_y[k]; }
    return s->np;
}

long orc_step_count(const orc_sim *s) { return s->step; }

/* Evaluate the thermal right-hand side L(Y) for a caller-given stage field Y using the frozen
 * rho, u of the current state (test hook for the discrete operator). */
int orc_thermal_rhs(orc_sim *s, const double *Y, double *L)
{
    current_fields(s);
    thermal_frozen(s);
    double *Yc = alloc_d((size_t)s->n);
    for (int k = 0; k < s->n; ++k) Yc[k] = s->solid[k] ? s->T_w : Y[k];
    thermal_rhs(s, Yc, L);
    free(Yc);
    return 0;
}


/* One Runge-Kutta update of a caller-given temperature field Y with the frozen rho, u of the
 * current state (test hook for the time integrator); writes the result to out. */
int orc_thermal_advance(orc_sim *s, const double *Y, double *out)
{
    current_fields(s);
    double *saved = alloc_d((size_t)s->n);
    memcpy(saved, s->T, sizeof(double) * (size_t)s->n);
    for (int k = 0; k < s->n; ++k) s->T[k] = s->solid[k] ? s->T_w : Y[k];
    thermal_update(s);
    memcpy(out, s->T, sizeof(double) * (size_t)s->n);
    memcpy(s->T, saved, sizeof(double) * (size_t)s->n);
    free(saved);
    return 0;
}

/* Isotropic-stencil operators on a periodic field (test hooks, same stencil as the force) */
void orc_iso_grad_periodic(int nx, int ny, const double *a, double *gx, double *gy)
{
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double sx = 0, sy = 0;
            for (int ey = -2; ey <= 2; ++ey)
                for (int ex = -2; ex <= 2; ++ex) {
                    if (ex == 0 && ey == 0) continue;
                    double w = stencil_w(ex * ex + ey * ey);
                    double v = a[wrapi(y + ey, ny) * nx + wrapi(x + ex, nx)];
                    sx += w * v * ex;
                    sy += w * v * ey;
                }
            gx[y * nx + x] = sx;
            gy[y * nx + x] = sy;
        }
}

void orc_iso_lap_periodic(int nx, int ny, const double *a, double *lap)
{
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double s = 0, a0 = a[y * nx + x];
            for (int ey = -2; ey <= 2; ++ey)
                for (int ex = -2; ex <= 2; ++ex) {
                    if (ex == 0 && ey == 0) continue;
                    s += 2.0 * stencil_w(ex * ex + ey * ey) * (a[wrapi(y + ey, ny) * nx + wrapi(x + ex, nx)] - a0);
                }
            lap[y * nx + x] = s;
        }
}

double orc_stencil_weight(int e2) { return stencil_w(e2); }

/* number of threads the OpenMP loops over nodes use */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
