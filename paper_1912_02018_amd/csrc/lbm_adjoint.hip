// Reverse-mode (adjoint) differentiation of one coupled FP64 step of the central-moment
// pseudopotential LBM with the finite-difference temperature equation (Saito et al.,
// arXiv:1912.02018, Sec. II and IV), with respect to the wall superheat, the inlet velocity, the
// acentric factor of the Peng-Robinson EOS and the relaxation time, for an objective built from the
// wall Nusselt number of Sec. IV B.
//
// Given the state n of a run (post-collision populations f*, outlet history, temperature T^n) and
// the adjoint of the state n+1 (lambda_f*, lambda_hist, lambda_T and the accumulated parameter
// gradient), one adjoint step
//   1. recomputes the forward step from state n, keeping its intermediates in scratch planes:
//      streamed populations, rho, j, psi, the interaction-stencil sums G, the force, u, the frozen
//      thermal fields grad(rho), div(u), the coefficients of the temperature operator and the
//      Runge-Kutta stage inputs;
//   2. runs the reverse of every stage of the step in the opposite order: the Runge-Kutta stages
//      (transposed temperature stencil), the coefficients of the temperature operator, the frozen
//      gradient / divergence stencils, this step's Nu sample, the collision, the interaction force
//      and the pseudopotential, the boundary conditions and the streaming;
//   3. reduces the parameter contributions of the step in a fixed order.
// Stencil transposes are written out by hand in gather form (every node sums what it fed into its
// neighbours, so no atomics and the result is reproducible bit for bit).  The Jacobians of the
// node-local maps (collision, pseudopotential, coefficients of the temperature operator, the
// equilibrium) are applied by evaluating those maps once more in forward-mode dual numbers (the
// same functions the step kernels use), seeded along the node's inputs or along the parameters.
//
// Supported: FP64 runs, x periodic or velocity inlet / convective outlet at speed u_in, constant
// transport properties, RK2 or RK4 or no temperature update, any warm-up, nx and ny >= 5.
// The kernels are plain global-memory node kernels (one thread per node): this is a sensitivity
// tool, run for thousands of steps on one grid, not the throughput path.

#include "lbm_device.h"

namespace lbm {
namespace {

// ---- scratch planes (FP64, [ny][pitch] each) ------------------------------------------------
enum {
    PF = 0,                                            // streamed populations f_i [9]
    PRHO = 9, PJX, PJY, PPSI, PGX, PGY, PFX, PFY, PA, PU, PV,
    PRX, PRY, PDIV,                                    // frozen thermal fields: grad rho, div u
    PCU12, PCV12, PCAU, PCAV, PCGX, PCGY, PCC0, PCC2,  // coefficients of the temperature operator
    PY2, PY3, PY4,                                     // Runge-Kutta stage inputs (Y1 = T^n)
    PKB0, PKB1,                                        // adjoints of the stage slopes (ping-pong)
    PBU12, PBV12, PBAU, PBAV, PBCGX, PBCGY, PBC0, PBC2, PBLAP,  // adjoints of the coefficients
    PBRX, PBRY, PBDIV,                                 // adjoints of the frozen fields
    PBRHO, PBU, PBV, PBT,                              // adjoints of rho, u, v, T^n
    PBPSI, PBGX, PBGY,                                 // adjoints of psi (local part) and G
    PBF,                                               // adjoints of the streamed populations [9]
    PTH = PBF + 9,                                     // per-node parameter contributions [4]
    NPLANES = PTH + kTangents
};
// after the planes: probe values [kMaxProbes][2], then the probes' parameter contribution [4], then
// the partial sums of the per-node parameter contributions [kThetaBlocks][4]
constexpr int kThetaBlocks = 256;

struct AdjArgs {
    const double *fs, *hist, *T;   // state n
    const double *ain;             // adjoint of state n+1
    double *aout;                  // adjoint of state n
    double *ws;                    // scratch planes
    long long step;                // n
    double wJ;                     // dJ / dNu of this step's Nu sample (0: none)
    int stage;                     // stage of the stage kernels
    int fon, thermal;              // forcing / temperature update active in this step
};

__device__ inline size_t plane_of(const RunDev &R) { return (size_t)R.ny * R.pitch; }
__device__ inline double *PL(const AdjArgs &a, const RunDev &R, int k) { return a.ws + (size_t)k * plane_of(R); }
__device__ inline size_t nid(const RunDev &R, int x, int y) { return (size_t)y * R.pitch + x; }
__device__ inline double *probe_vals(const AdjArgs &a, const RunDev &R) { return a.ws + (size_t)NPLANES * plane_of(R); }
__device__ inline double *probe_theta(const AdjArgs &a, const RunDev &R) { return probe_vals(a, R) + 2 * kMaxProbes; }
__device__ inline double *theta_parts(const AdjArgs &a, const RunDev &R) { return probe_theta(a, R) + kTangents; }
// workgroups of the parameter-contribution sum: row blocks of about equal height
__host__ __device__ inline int theta_blocks(int ny) { return ny < kThetaBlocks ? ny : kThetaBlocks; }

// adjoint state layout: lambda_f* [9] planes, lambda_T plane, lambda_hist [3][ny], dJ/dtheta [4]
__device__ inline size_t adj_T(const RunDev &R) { return 9 * plane_of(R); }
__device__ inline size_t adj_hist(const RunDev &R) { return 10 * plane_of(R); }
__device__ inline size_t adj_theta(const RunDev &R) { return 10 * plane_of(R) + 3 * (size_t)R.ny; }

// weight w(|e|^2) of the interaction stencil (eq. interForce)
__device__ inline double stencil_w(int ex, int ey)
{
    switch (ex * ex + ey * ey) {
    case 1: return W1;
    case 2: return W2;
    case 4: return W4;
    case 5: return W5;
    case 8: return W8;
    default: return 0.0;
    }
}

__device__ inline bool node_kernel_index(const RunDev &R, int &x, int &y)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (long long)R.nx * R.ny) return false;
    x = (int)(k % R.nx);
    y = (int)(k / R.nx);
    return true;
}

// wrapped row difference t - s in [-2, 2] (ny >= 5: unique)
__device__ inline int row_offset(int ty, int sy, int ny)
{
    int d = ty - sy;
    if (d > 2) d -= ny;
    if (d < -2) d += ny;
    return d;
}

// Gather helper: calls fn(sx, sy, ex, ey) for every domain node s = (sx, sy) and stencil offset
// e != 0 whose extended position s + e carries the value of node t (the node itself through the
// periodic wraps; at the outlet column the outlet ghosts; with inlet_copies, at the inlet column the
// inlet ghosts, which copy column 0 for rho and u but not for psi or the temperature).
template <typename Fn>
__device__ inline void for_sources(const RunDev &R, int tx, int ty, bool inlet_copies, Fn fn)
{
    const int nx = R.nx, ny = R.ny;
    for (int dy = -2; dy <= 2; ++dy) {
        const int sy = wrap(ty + dy, ny);
        const int ey = row_offset(ty, sy, ny);
        for (int dx = -2; dx <= 2; ++dx) {
            int sx = tx + dx;
            if (R.bc_x == 0) sx = wrap(sx, nx);
            else if (sx < 0 || sx >= nx) continue;
            for (int ex = -2; ex <= 2; ++ex) {
                if (ex == 0 && ey == 0) continue;
                const int px = sx + ex;
                bool hit;
                if (R.bc_x == 0) hit = wrap(px, nx) == tx;
                else hit = px == tx || (tx == nx - 1 && px >= nx) || (inlet_copies && tx == 0 && px < 0);
                if (hit) fn(sx, sy, ex, ey);
            }
        }
    }
}

// value of a node field at an extended position for rho / u (inlet ghosts copy column 0, outlet
// ghosts column nx-1)
__device__ inline double ext_copy(const RunDev &R, const double *f, int gx, int gy)
{
    int rx, ry;
    map_pos<false>(R, gx, gy, rx, ry);
    return f[nid(R, rx, ry)];
}

// ---- node-local maps, templated on the scalar type ------------------------------------------
// coefficients of the temperature operator at a fluid node (constant transport properties):
// c[0..7] = u/12, v/12, |u| c_d, |v| c_d, (alpha/rho) d_x rho, (alpha/rho) d_y rho, centre, sqrt term
template <typename C>
__device__ inline void thermal_coef(const Consts<C> &K, double cd, C rho, C Rx, C Ry, C u, C v, C div, C c[8])
{
    const C ir = Ar<C>::rcp(rho);
    const C gcoef = K.alpha * ir;
    const C D = div * ir * K.inv_cv;
    const C d1 = (C)1 - K.b * rho;
    const C d2 = (C)1 + (C)2 * K.b * rho - K.b * K.b * rho * rho;
    const C A2 = D * K.a * rho * rho * Ar<C>::rcp(d2);
    const C c1 = -D * rho * K.Rg * Ar<C>::rcp(d1) + K.dphi_B * A2;
    const C au = absval(u) * (C)cd, av = absval(v) * (C)cd;
    c[0] = u * (C)(1.0 / 12.0);
    c[1] = v * (C)(1.0 / 12.0);
    c[2] = au;
    c[3] = av;
    c[4] = gcoef * Rx;
    c[5] = gcoef * Ry;
    c[6] = c1 - (C)(2 * WSUM) * K.alpha - (C)6 * (au + av);
    c[7] = K.dphi_A * A2;
}

// density, momentum and raw second moments of a population set (the order of the step kernel)
template <typename C> __device__ inline void raw_moments(const C f[9], C &rho, C &jx, C &jy, C &m4, C &m5)
{
    rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    jx = (f[1] - f[2]) + (f[5] - f[6]) + (f[7] - f[8]);
    jy = (f[3] - f[4]) + (f[5] - f[6]) + (f[8] - f[7]);
    m4 = (f[1] + f[2]) - (f[3] + f[4]);
    m5 = (f[5] + f[6]) - (f[7] + f[8]);
}

// full Hermite equilibrium (eq. equi), as the initial state takes it
template <typename C> __device__ inline void equilibrium(C r, C u, C v, C feq[9])
{
    const C cs2 = (C)(1.0 / 3.0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const C cx = (C)cx_of(i), cy = (C)cy_of(i);
        const C H2xx = cx * cx - cs2, H2yy = cy * cy - cs2, H2xy = cx * cy;
        const C H3xxy = (cx * cx - cs2) * cy, H3xyy = cx * (cy * cy - cs2);
        const C H4 = (cx * cx - cs2) * (cy * cy - cs2);
        const C t1 = (cx * u + cy * v) / cs2;
        const C t2 = (H2xx * u * u + (C)2 * H2xy * u * v + H2yy * v * v) / ((C)2 * cs2 * cs2);
        const C t3 = (H3xxy * u * u * v + H3xyy * u * v * v) / ((C)2 * cs2 * cs2 * cs2);
        const C t4 = H4 * u * u * v * v / ((C)4 * cs2 * cs2 * cs2 * cs2);
        feq[i] = (C)lat_w(i) * r * ((C)1 + t1 + t2 + t3 + t4);
    }
}

__device__ inline Dual seed(double v, int k)
{
    Dual r(v);
    r.d[k] = 1.0;
    return r;
}

__device__ inline void add_theta(double *th, size_t plane, size_t i, const double g[kTangents])
{
#pragma unroll
    for (int k = 0; k < kTangents; ++k) th[(size_t)k * plane + i] += g[k];
}

// window quantities of the temperature operator at (x, y) on a stage field Y (ghosts: inlet T_sat,
// outlet the last column, solid nodes their held value)
struct Win {
    double lapw, gx, gy, cx1, sx, cy1, sy, y0;
};
__device__ inline double ext_Y(const RunDev &R, const double *Y, int gx, int gy)
{
    int rx, ry;
    const int kind = map_pos<false>(R, gx, gy, rx, ry);
    return kind == INLET_GHOST ? R.T_sat : Y[nid(R, rx, ry)];
}
// a node whose 5 x 5 window holds no ghost position (x two columns from an inlet or outlet; any x with
// periodic columns, nx >= 5): its stencil positions and sources are plain offsets (rows wrap)
__device__ inline bool plain_columns(const RunDev &R, int x) { return R.bc_x == 0 || (x >= 2 && x <= R.nx - 3); }
__device__ inline int wrap_col(const RunDev &R, int x) { return R.bc_x == 0 ? wrap(x, R.nx) : x; }
__device__ inline Win window(const RunDev &R, const double *Y, int x, int y)
{
    if (plain_columns(R, x)) {
        // the same sums in the same order, without the ghost mapping of every position
        Win w{0, 0, 0, 0, 0, 0, 0, 0};
        w.y0 = Y[nid(R, x, y)];
        double v[5][5];
#pragma unroll
        for (int ey = -2; ey <= 2; ++ey) {
            const int yy = wrap(y + ey, R.ny);
#pragma unroll
            for (int ex = -2; ex <= 2; ++ex) v[ey + 2][ex + 2] = Y[nid(R, wrap_col(R, x + ex), yy)];
        }
#pragma unroll
        for (int ey = -2; ey <= 2; ++ey)
#pragma unroll
            for (int ex = -2; ex <= 2; ++ex) {
                if (ex == 0 && ey == 0) continue;
                const double yv = v[ey + 2][ex + 2], we = stencil_w(ex, ey);
                w.lapw += 2.0 * we * yv;
                w.gx += we * ex * yv;
                w.gy += we * ey * yv;
            }
        const double xp1 = v[2][3], xm1 = v[2][1], xp2 = v[2][4], xm2 = v[2][0];
        const double yp1 = v[3][2], ym1 = v[1][2], yp2 = v[4][2], ym2 = v[0][2];
        w.cx1 = 8.0 * (xp1 - xm1) - (xp2 - xm2);
        w.sx = (xp2 + xm2) - 4.0 * (xp1 + xm1);
        w.cy1 = 8.0 * (yp1 - ym1) - (yp2 - ym2);
        w.sy = (yp2 + ym2) - 4.0 * (yp1 + ym1);
        return w;
    }
    Win w{0, 0, 0, 0, 0, 0, 0, 0};
    w.y0 = Y[nid(R, x, y)];
    for (int ey = -2; ey <= 2; ++ey)
        for (int ex = -2; ex <= 2; ++ex) {
            if (ex == 0 && ey == 0) continue;
            const double yv = ext_Y(R, Y, x + ex, y + ey), we = stencil_w(ex, ey);
            w.lapw += 2.0 * we * yv;
            w.gx += we * ex * yv;
            w.gy += we * ey * yv;
        }
    const double xp1 = ext_Y(R, Y, x + 1, y), xm1 = ext_Y(R, Y, x - 1, y);
    const double xp2 = ext_Y(R, Y, x + 2, y), xm2 = ext_Y(R, Y, x - 2, y);
    const double yp1 = ext_Y(R, Y, x, y + 1), ym1 = ext_Y(R, Y, x, y - 1);
    const double yp2 = ext_Y(R, Y, x, y + 2), ym2 = ext_Y(R, Y, x, y - 2);
    w.cx1 = 8.0 * (xp1 - xm1) - (xp2 - xm2);
    w.sx = (xp2 + xm2) - 4.0 * (xp1 + xm1);
    w.cy1 = 8.0 * (yp1 - ym1) - (yp2 - ym2);
    w.sy = (yp2 + ym2) - 4.0 * (yp1 + ym1);
    return w;
}
// L(Y) at a fluid node with coefficients c
__device__ inline double apply_L(double alpha, const double c[8], const Win &w)
{
    return alpha * w.lapw - (c[0] * w.cx1 + c[2] * w.sx + c[1] * w.cy1 + c[3] * w.sy) + c[4] * w.gx + c[5] * w.gy +
           c[6] * w.y0 + c[7] * sqrt(w.y0);
}
// weight a_e(s) with which L at node s takes its stencil position s + e (e != 0)
__device__ inline double stencil_coef(double alpha, const double c[8], int ex, int ey)
{
    const double we = stencil_w(ex, ey);
    double a = 2.0 * alpha * we + c[4] * we * ex + c[5] * we * ey;
    if (ey == 0) {
        if (ex == 1) a += -8.0 * c[0] + 4.0 * c[2];
        else if (ex == -1) a += 8.0 * c[0] + 4.0 * c[2];
        else if (ex == 2) a += c[0] - c[2];
        else if (ex == -2) a += -c[0] - c[2];
    }
    if (ex == 0) {
        if (ey == 1) a += -8.0 * c[1] + 4.0 * c[3];
        else if (ey == -1) a += 8.0 * c[1] + 4.0 * c[3];
        else if (ey == 2) a += c[1] - c[3];
        else if (ey == -2) a += -c[1] - c[3];
    }
    return a;
}
__device__ inline void load_coef(const AdjArgs &a, const RunDev &R, size_t i, double c[8])
{
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = PL(a, R, PCU12 + k)[i];
}
__device__ inline double stage_a(int NS, int s) { return NS == 4 ? (s == 3 ? 1.0 : 0.5) : 1.0; }   // Y_{s+1} = T + a_s k_s
__device__ inline double stage_b(int NS, int s) { return NS == 4 ? ((s == 1 || s == 4) ? 1.0 / 6.0 : 1.0 / 3.0) : 0.5; }
__device__ inline const double *stage_Y(const AdjArgs &a, const RunDev &R, int s)
{
    return s == 1 ? a.T : PL(a, R, PY2 + (s - 2));
}

// ============================================================================================
// Forward recompute
// ============================================================================================
// streaming with the boundary conditions; rho, j
__global__ __launch_bounds__(256) void ka_stream(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    const size_t P = plane_of(R), i0 = nid(R, x, y);
    double f[9];
    if (solid_at(R, x, y)) {
        for (int i = 0; i < 9; ++i) PL(a, R, PF + i)[i0] = 0.0;
        PL(a, R, PRHO)[i0] = R.rho_w;
        PL(a, R, PJX)[i0] = 0.0;
        PL(a, R, PJY)[i0] = 0.0;
        return;
    }
    const int bw = 2 * R.cyl_r + 3;
    for (int i = 0; i < 9; ++i) {
        int xs = x - cx_of(i);
        const int ys = wrap(y - cy_of(i), R.ny);
        if (R.bc_x == 0) xs = wrap(xs, R.nx);
        else if (xs < 0 || xs >= R.nx) { f[i] = 0.0; continue; }
        if (!solid_at(R, xs, ys)) { f[i] = a.fs[(size_t)i * P + nid(R, xs, ys)]; continue; }
        // interpolated bounce-back (wall fraction table of the cut links)
        const int o = opp_of(i);
        const double v = ((const double *)R.qtab)[((y - (R.cyl_y - R.cyl_r - 1)) * bw + (x - (R.cyl_x - R.cyl_r - 1))) * 8 + (i - 1)];
        const double fo = a.fs[(size_t)o * P + i0];
        if (v > 2.0) f[i] = fo;
        else if (v > 0.0) f[i] = v * fo + (1.0 - v) * a.fs[(size_t)o * P + nid(R, x + cx_of(i), wrap(y + cy_of(i), R.ny))];
        else { const double q2 = -v; f[i] = fo / q2 + (q2 - 1.0) / q2 * a.fs[(size_t)i * P + i0]; }
    }
    if (R.bc_x == 1 && x == R.nx - 1) {
        const double U = R.u_in;
        const int dirs[3] = {2, 6, 8};
        for (int m = 0; m < 3; ++m) {
            const int i = dirs[m];
            const double p = a.fs[(size_t)i * P + nid(R, R.nx - 1, wrap(y - cy_of(i), R.ny))];
            f[i] = (a.hist[m * R.ny + y] + U * p) / (1.0 + U);
        }
    }
    if (R.bc_x == 1 && x == 0) {
        const double u = R.u_in;
        const double rin = (f[0] + f[3] + f[4] + 2.0 * (f[2] + f[6] + f[8])) / (1.0 - u);
        f[1] = f[2] + (2.0 / 3.0) * rin * u;
        f[5] = f[6] - 0.5 * (f[3] - f[4]) + rin * u / 6.0;
        f[7] = f[8] + 0.5 * (f[3] - f[4]) + rin * u / 6.0;
    }
    double rho, jx, jy, m4, m5;
    raw_moments(f, rho, jx, jy, m4, m5);
    for (int i = 0; i < 9; ++i) PL(a, R, PF + i)[i0] = f[i];
    PL(a, R, PRHO)[i0] = rho;
    PL(a, R, PJX)[i0] = jx;
    PL(a, R, PJY)[i0] = jy;
}

// pseudopotential at every node (solid nodes: rho_w, T_w)
__global__ __launch_bounds__(256) void ka_psi(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    const Consts<double> K(R);
    const size_t i0 = nid(R, x, y);
    PL(a, R, PPSI)[i0] = solid_at(R, x, y) ? pseudopotential(K, K.rho_w, K.T_w)
                                           : pseudopotential(K, PL(a, R, PRHO)[i0], a.T[i0]);
}

// psi on the extended field
__device__ inline double ext_psi(const AdjArgs &a, const RunDev &R, const Consts<double> &K, int gx, int gy)
{
    int rx, ry;
    const int kind = map_pos<false>(R, gx, gy, rx, ry);
    if (kind == INLET_GHOST) return pseudopotential(K, PL(a, R, PRHO)[nid(R, rx, ry)], K.T_sat);
    return PL(a, R, PPSI)[nid(R, rx, ry)];
}

// interaction-stencil sums G, force, consistency term, velocity
__global__ __launch_bounds__(256) void ka_force(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    const Consts<double> K(R);
    const size_t i0 = nid(R, x, y);
    double Gx = 0, Gy = 0, Fx = 0, Fy = 0, A = 0, U = 0, V = 0;
    if (!solid_at(R, x, y)) {
        const double rho = PL(a, R, PRHO)[i0];
        if (a.fon) {
            for (int ey = -2; ey <= 2; ++ey)
                for (int ex = -2; ex <= 2; ++ex) {
                    if (ex == 0 && ey == 0) continue;
                    const double ps = ext_psi(a, R, K, x + ex, y + ey), we = stencil_w(ex, ey);
                    Gx += we * ex * ps;
                    Gy += we * ey * ps;
                }
            const double psi0 = PL(a, R, PPSI)[i0];
            const double pre = -2.0 / K.psi_scale * psi0;
            const double Fmx = pre * Gx, Fmy = pre * Gy;
            A = 2.0 * K.sigma * (Fmx * Fmx + Fmy * Fmy) / (psi0 * psi0);
            Fx = Fmx + (rho - K.rho_gref) * K.gx;
            Fy = Fmy + (rho - K.rho_gref) * K.gy;
        }
        const double ir = 1.0 / rho;
        U = (PL(a, R, PJX)[i0] + 0.5 * Fx) * ir;
        V = (PL(a, R, PJY)[i0] + 0.5 * Fy) * ir;
    }
    PL(a, R, PGX)[i0] = Gx;
    PL(a, R, PGY)[i0] = Gy;
    PL(a, R, PFX)[i0] = Fx;
    PL(a, R, PFY)[i0] = Fy;
    PL(a, R, PA)[i0] = A;
    PL(a, R, PU)[i0] = U;
    PL(a, R, PV)[i0] = V;
}

// frozen thermal fields and the coefficients of the temperature operator
__global__ __launch_bounds__(256) void ka_frozen(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    const Consts<double> K(R);
    const size_t i0 = nid(R, x, y);
    double Rx = 0, Ry = 0, dv = 0, c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (!solid_at(R, x, y)) {
        const double *rho = PL(a, R, PRHO), *u = PL(a, R, PU), *v = PL(a, R, PV);
        for (int ey = -2; ey <= 2; ++ey)
            for (int ex = -2; ex <= 2; ++ex) {
                if (ex == 0 && ey == 0) continue;
                const double we = stencil_w(ex, ey);
                Rx += we * ex * ext_copy(R, rho, x + ex, y + ey);
                Ry += we * ey * ext_copy(R, rho, x + ex, y + ey);
                dv += we * (ex * ext_copy(R, u, x + ex, y + ey) + ey * ext_copy(R, v, x + ex, y + ey));
            }
        thermal_coef<double>(K, R.upwind_kind == 1 ? 0.25 : 1.0 / 12.0, rho[i0], Rx, Ry, u[i0], v[i0], dv, c);
    }
    PL(a, R, PRX)[i0] = Rx;
    PL(a, R, PRY)[i0] = Ry;
    PL(a, R, PDIV)[i0] = dv;
    for (int k = 0; k < 8; ++k) PL(a, R, PCU12 + k)[i0] = c[k];
}

// stage input Y_{s+1} = T + a_s L(Y_s) (held nodes keep T)
__global__ __launch_bounds__(256) void ka_stage(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    const size_t i0 = nid(R, x, y);
    const int s = a.stage;
    double out = a.T[i0];
    if (!solid_at(R, x, y)) {
        double c[8];
        load_coef(a, R, i0, c);
        out += stage_a(R.rk, s) * apply_L(R.alpha, c, window(R, stage_Y(a, R, s), x, y));
    }
    PL(a, R, PY2 + (s - 1))[i0] = out;
}

// ============================================================================================
// Reverse
// ============================================================================================
// clear the accumulators; the adjoint of T^{n+1} enters: T^{n+1} = T^n + sum_s b_s k_s at fluid
// nodes, T_w at solid nodes (the superheat), T^n everywhere when the step does not update T
__global__ __launch_bounds__(256) void kb_init(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    const size_t P = plane_of(R), i0 = nid(R, x, y);
    for (int k = PBU12; k < NPLANES; ++k) PL(a, R, k)[i0] = 0.0;
    const double tb = a.ain[adj_T(R) + i0];
    if (!a.thermal) {
        PL(a, R, PBT)[i0] = tb;
        return;
    }
    if (solid_at(R, x, y)) {
        double g[kTangents];
        for (int k = 0; k < kTangents; ++k) g[k] = tb * R.t_T_w[k];
        add_theta(PL(a, R, PTH), P, i0, g);
        PL(a, R, PKB0 + (R.rk & 1))[i0] = 0.0;
        return;
    }
    PL(a, R, PBT)[i0] = tb;
    PL(a, R, PKB0 + (R.rk & 1))[i0] = stage_b(R.rk, R.rk) * tb;
}

// reverse of stage s: with kbar_s (plane (s & 1)) complete, every node
//   * accumulates the adjoints of its coefficients, kbar_s dL/dcoef on Y_s;
//   * gathers Ybar_s = L_Y^T kbar_s (transposed stencil; centre with the sqrt term's derivative);
//   * adds Ybar_s to the adjoint of T^n (Y_s = T^n + a k_{s-1}, held nodes Y_s = T^n);
//   * forms kbar_{s-1} = b_{s-1} Tbar' + a_{s-1} Ybar_s (fluid nodes) in the other plane.
__global__ __launch_bounds__(256) void kb_stage(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    const size_t i0 = nid(R, x, y);
    const int s = a.stage;
    const double *kb = PL(a, R, PKB0 + (s & 1));
    const double *Y = stage_Y(a, R, s);
    const bool fluid = !solid_at(R, x, y);
    if (fluid) {
        const double k = kb[i0];
        const Win w = window(R, Y, x, y);
        PL(a, R, PBU12)[i0] -= k * w.cx1;
        PL(a, R, PBV12)[i0] -= k * w.cy1;
        PL(a, R, PBAU)[i0] -= k * w.sx;
        PL(a, R, PBAV)[i0] -= k * w.sy;
        PL(a, R, PBCGX)[i0] += k * w.gx;
        PL(a, R, PBCGY)[i0] += k * w.gy;
        PL(a, R, PBC0)[i0] += k * w.y0;
        PL(a, R, PBC2)[i0] += k * sqrt(w.y0);
        PL(a, R, PBLAP)[i0] += k * w.lapw;
    }
    double yb = 0.0;
    auto source = [&](int sx, int sy, int ex, int ey) {
        if (solid_at(R, sx, sy)) return;
        double c[8];
        const size_t is = nid(R, sx, sy);
        load_coef(a, R, is, c);
        yb += stencil_coef(R.alpha, c, ex, ey) * kb[is];
    };
    if (plain_columns(R, x)) {
        // the sources t - e in for_sources' order, with compile-time offsets (so that only the
        // coefficients a source's offset uses are loaded)
#pragma unroll
        for (int dy = -2; dy <= 2; ++dy) {
            const int sy = wrap(y + dy, R.ny);
#pragma unroll
            for (int dx = -2; dx <= 2; ++dx)
                if (dx != 0 || dy != 0) source(wrap_col(R, x + dx), sy, -dx, -dy);
        }
    } else {
        for_sources(R, x, y, false, source);
    }
    if (fluid) {
        double c[8];
        load_coef(a, R, i0, c);
        yb += (c[6] + c[7] * 0.5 / sqrt(Y[i0])) * kb[i0];
    }
    PL(a, R, PBT)[i0] += yb;
    if (s > 1) {
        const double tb = a.ain[adj_T(R) + i0];
        PL(a, R, PKB0 + ((s - 1) & 1))[i0] = fluid ? stage_b(R.rk, s - 1) * tb + stage_a(R.rk, s - 1) * yb : 0.0;
    }
}

// coefficient adjoints -> adjoints of rho, grad rho, u, v, div u and of the parameters (local
// Jacobian of thermal_coef in dual numbers)
__global__ __launch_bounds__(256) void kb_coef(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    if (solid_at(R, x, y)) return;
    const size_t P = plane_of(R), i0 = nid(R, x, y);
    const double cd = R.upwind_kind == 1 ? 0.25 : 1.0 / 12.0;
    double cb[8];
    for (int k = 0; k < 8; ++k) cb[k] = PL(a, R, PBU12 + k)[i0];
    const double in[6] = {PL(a, R, PRHO)[i0], PL(a, R, PRX)[i0], PL(a, R, PRY)[i0],
                          PL(a, R, PU)[i0],   PL(a, R, PV)[i0],  PL(a, R, PDIV)[i0]};
    double bar[6] = {0, 0, 0, 0, 0, 0};
    const Consts<Dual> Ku(R, false);
    for (int pass = 0; pass < 2; ++pass) {
        Dual d[6];
        for (int j = 0; j < 6; ++j) {
            d[j] = Dual(in[j]);
            const int slot = j - 4 * pass;
            if (slot >= 0 && slot < 4) d[j].d[slot] = 1.0;
        }
        Dual c[8];
        thermal_coef<Dual>(Ku, cd, d[0], d[1], d[2], d[3], d[4], d[5], c);
        for (int j = 4 * pass; j < 6 && j < 4 * pass + 4; ++j)
            for (int k = 0; k < 8; ++k) bar[j] += cb[k] * c[k].d[j - 4 * pass];
    }
    // parameters: the coefficients' own dependence, and alpha of the Laplacian (dL/dalpha = lapw)
    {
        const Consts<Dual> Ks(R, true);
        Dual c[8];
        thermal_coef<Dual>(Ks, cd, Dual(in[0]), Dual(in[1]), Dual(in[2]), Dual(in[3]), Dual(in[4]), Dual(in[5]), c);
        double g[kTangents];
        const double blap = PL(a, R, PBLAP)[i0];
        for (int t = 0; t < kTangents; ++t) {
            g[t] = blap * R.t_alpha[t];
            for (int k = 0; k < 8; ++k) g[t] += cb[k] * c[k].d[t];
        }
        add_theta(PL(a, R, PTH), P, i0, g);
    }
    PL(a, R, PBRHO)[i0] += bar[0];
    PL(a, R, PBRX)[i0] = bar[1];
    PL(a, R, PBRY)[i0] = bar[2];
    PL(a, R, PBU)[i0] += bar[3];
    PL(a, R, PBV)[i0] += bar[4];
    PL(a, R, PBDIV)[i0] = bar[5];
}

// transposed gradient / divergence stencils of the frozen fields (rho and u of solid nodes are
// constants; inlet ghosts copy column 0, outlet ghosts column nx-1)
__global__ __launch_bounds__(256) void kb_frozen_gather(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    if (solid_at(R, x, y)) return;
    const size_t i0 = nid(R, x, y);
    double rb = 0, ub = 0, vb = 0;
    for_sources(R, x, y, true, [&](int sx, int sy, int ex, int ey) {
        if (solid_at(R, sx, sy)) return;
        const size_t is = nid(R, sx, sy);
        const double we = stencil_w(ex, ey), db = PL(a, R, PBDIV)[is];
        rb += we * (ex * PL(a, R, PBRX)[is] + ey * PL(a, R, PBRY)[is]);
        ub += we * ex * db;
        vb += we * ey * db;
    });
    PL(a, R, PBRHO)[i0] += rb;
    PL(a, R, PBU)[i0] += ub;
    PL(a, R, PBV)[i0] += vb;
}

// this step's Nu sample: bilinear rho and T at the probes (one workgroup, fixed order), and the
// explicit superheat dependence of Nu = 2R / (1.5 N_p rho_v dT) sum_p rho_p (T_w - T_p)
__global__ __launch_bounds__(256) void kb_probe(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    __shared__ double red[256];
    double *pv = probe_vals(a, R);
    double sr = 0.0, snu = 0.0;
    for (int k = threadIdx.x; k < R.np; k += 256) {
        const double px = R.probes[2 * k], py = R.probes[2 * k + 1];
        const int x0 = (int)floor(px), y0 = (int)floor(py);
        const double fx = px - x0, fy = py - y0;
        const double w00 = (1 - fx) * (1 - fy), w10 = fx * (1 - fy), w01 = (1 - fx) * fy, w11 = fx * fy;
        const double *rho = PL(a, R, PRHO);
        const size_t i00 = nid(R, x0, y0), i01 = i00 + R.pitch;
        const double r = w00 * rho[i00] + w10 * rho[i00 + 1] + w01 * rho[i01] + w11 * rho[i01 + 1];
        const double t = w00 * a.T[i00] + w10 * a.T[i00 + 1] + w01 * a.T[i01] + w11 * a.T[i01 + 1];
        pv[2 * k] = r;
        pv[2 * k + 1] = t;
        sr += r;
        snu += r * (R.T_w - t);
    }
    for (int pass = 0; pass < 2; ++pass) {
        red[threadIdx.x] = pass == 0 ? sr : snu;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (pass == 0) sr = red[0];
        else snu = red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double dT = R.T_w - R.T_sat;
        const double Cn = 2.0 * R.cyl_r / (1.5 * R.np * R.rho_v * dT);
        const double nu = Cn * snu;
        const double dnu = Cn * sr - nu / dT;   // d Nu / d T_w at fixed fields
        double *th = probe_theta(a, R);
        for (int k = 0; k < kTangents; ++k) th[k] = a.wJ * dnu * R.t_T_w[k];
    }
}

// adjoints of rho and T^n from the Nu sample (each node sums its probes' bilinear weights)
__global__ __launch_bounds__(256) void kb_nu(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    const int reach = R.cyl_r + 3;
    if (abs(x - R.cyl_x) > reach || abs(y - R.cyl_y) > reach) return;
    const size_t i0 = nid(R, x, y);
    const double dT = R.T_w - R.T_sat;
    const double Cn = a.wJ * 2.0 * R.cyl_r / (1.5 * R.np * R.rho_v * dT);
    const double *pv = probe_vals(a, R);
    double rb = 0, tb = 0;
    for (int k = 0; k < R.np; ++k) {
        const double px = R.probes[2 * k], py = R.probes[2 * k + 1];
        const int x0 = (int)floor(px), y0 = (int)floor(py);
        if (x < x0 || x > x0 + 1 || y < y0 || y > y0 + 1) continue;
        const double fx = px - x0, fy = py - y0;
        const double w = (x == x0 ? 1 - fx : fx) * (y == y0 ? 1 - fy : fy);
        rb += w * Cn * (R.T_w - pv[2 * k + 1]);
        tb -= w * Cn * pv[2 * k];
    }
    PL(a, R, PBRHO)[i0] += rb;
    PL(a, R, PBT)[i0] += tb;
}

// collision (and velocity) of a fluid node in reverse, through dual numbers: inputs f[9], F, A;
// outputs f*[9] (adjoint lambda_f* of state n+1) and u (adjoint from the temperature operator);
// then the interaction force F = c psi G + (rho - rho_gref) g, A = 2 sigma c^2 |G|^2 in reverse
__global__ __launch_bounds__(256) void kb_collide(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    if (solid_at(R, x, y)) return;
    const size_t P = plane_of(R), i0 = nid(R, x, y);
    double in[12], lout[11];
    for (int i = 0; i < 9; ++i) in[i] = PL(a, R, PF + i)[i0];
    in[9] = PL(a, R, PFX)[i0];
    in[10] = PL(a, R, PFY)[i0];
    in[11] = PL(a, R, PA)[i0];
    for (int i = 0; i < 9; ++i) lout[i] = a.ain[(size_t)i * P + i0];
    lout[9] = PL(a, R, PBU)[i0];
    lout[10] = PL(a, R, PBV)[i0];
    double bar[12];
    const Consts<Dual> Ku(R, false);
    for (int pass = 0; pass < 3; ++pass) {
        Dual d[12];
        for (int j = 0; j < 12; ++j) {
            d[j] = Dual(in[j]);
            if (j / 4 == pass) d[j].d[j % 4] = 1.0;
        }
        Dual rho, jx, jy, m4, m5, U, V, fs[9];
        raw_moments(d, rho, jx, jy, m4, m5);
        collide_node<Dual>(rho, jx, jy, m4, m5, d[9], d[10], d[11], Ku.omega, U, V, fs);
        for (int j = 4 * pass; j < 4 * pass + 4; ++j) {
            const int sl = j % 4;
            double b = lout[9] * U.d[sl] + lout[10] * V.d[sl];
            for (int i = 0; i < 9; ++i) b += lout[i] * fs[i].d[sl];
            bar[j] = b;
        }
    }
    {
        // the relaxation time: omega
        const Consts<Dual> Ks(R, true);
        Dual d[12];
        for (int j = 0; j < 12; ++j) d[j] = Dual(in[j]);
        Dual rho, jx, jy, m4, m5, U, V, fs[9];
        raw_moments(d, rho, jx, jy, m4, m5);
        collide_node<Dual>(rho, jx, jy, m4, m5, d[9], d[10], d[11], Ks.omega, U, V, fs);
        double g[kTangents];
        for (int t = 0; t < kTangents; ++t) {
            g[t] = 0.0;
            for (int i = 0; i < 9; ++i) g[t] += lout[i] * fs[i].d[t];
        }
        add_theta(PL(a, R, PTH), P, i0, g);
    }
    for (int i = 0; i < 9; ++i) PL(a, R, PBF + i)[i0] = bar[i];
    if (a.fon) {
        const double c = -2.0 / R.psi_scale, psi0 = PL(a, R, PPSI)[i0];
        const double Gx = PL(a, R, PGX)[i0], Gy = PL(a, R, PGY)[i0];
        const double Fbx = bar[9], Fby = bar[10], Ab = bar[11];
        PL(a, R, PBGX)[i0] = Fbx * c * psi0 + Ab * 4.0 * R.sigma * c * c * Gx;
        PL(a, R, PBGY)[i0] = Fby * c * psi0 + Ab * 4.0 * R.sigma * c * c * Gy;
        PL(a, R, PBPSI)[i0] = c * (Fbx * Gx + Fby * Gy);
        PL(a, R, PBRHO)[i0] += Fbx * R.gx + Fby * R.gy;
    }
}

// psi: transposed interaction stencil, then the EOS-consistent pseudopotential in reverse (its
// derivatives in rho, T and the parameters through dual numbers); solid nodes feed the parameters
// through psi(rho_w, T_w), inlet ghosts rho of column 0 through psi(rho, T_sat)
__global__ __launch_bounds__(256) void kb_psi(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    const size_t P = plane_of(R), i0 = nid(R, x, y);
    const bool solid = solid_at(R, x, y);
    double pb = solid ? 0.0 : PL(a, R, PBPSI)[i0];
    for_sources(R, x, y, false, [&](int sx, int sy, int ex, int ey) {
        if (solid_at(R, sx, sy)) return;
        const size_t is = nid(R, sx, sy);
        pb += stencil_w(ex, ey) * (ex * PL(a, R, PBGX)[is] + ey * PL(a, R, PBGY)[is]);
    });
    // inlet ghosts of this row (column 0 only): psi(rho(0, y), T_sat)
    double gb = 0.0;
    if (R.bc_x == 1 && x == 0) {
        for (int dy = -2; dy <= 2; ++dy) {
            const int sy = wrap(y + dy, R.ny), ey = row_offset(y, sy, R.ny);
            for (int sx = 0; sx <= 1; ++sx) {
                if (solid_at(R, sx, sy)) continue;
                const size_t is = nid(R, sx, sy);
                for (int ex = -2; ex <= 2; ++ex)
                    if (sx + ex < 0) gb += stencil_w(ex, ey) * (ex * PL(a, R, PBGX)[is] + ey * PL(a, R, PBGY)[is]);
            }
        }
    }
    const Consts<Dual> Ku(R, false), Ks(R, true);
    double g[kTangents] = {0, 0, 0, 0};
    if (solid) {
        const Dual ps = pseudopotential(Ks, Ks.rho_w, Ks.T_w);
        for (int t = 0; t < kTangents; ++t) g[t] = pb * ps.d[t];
    } else {
        const double rho = PL(a, R, PRHO)[i0], T = a.T[i0];
        const Dual pr = pseudopotential(Ku, seed(rho, 0), seed(T, 1));
        const Dual pt = pseudopotential(Ks, Dual(rho), Dual(T));
        PL(a, R, PBRHO)[i0] += pb * pr.d[0];
        PL(a, R, PBT)[i0] += pb * pr.d[1];
        for (int t = 0; t < kTangents; ++t) g[t] = pb * pt.d[t];
        if (gb != 0.0) {
            const Dual gr = pseudopotential(Ku, seed(rho, 0), Dual(R.T_sat));
            const Dual gt = pseudopotential(Ks, Dual(rho), Dual(R.T_sat));
            PL(a, R, PBRHO)[i0] += gb * gr.d[0];
            for (int t = 0; t < kTangents; ++t) g[t] += gb * gt.d[t];
        }
    }
    add_theta(PL(a, R, PTH), P, i0, g);
}

// adjoints of the streamed populations: collision part + rho (sum of f); the outlet history of
// state n+1, the convective outlet and the velocity inlet in reverse; writes lambda_hist of state n
__global__ __launch_bounds__(256) void kb_bc(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    if (solid_at(R, x, y)) return;
    const size_t P = plane_of(R), i0 = nid(R, x, y);
    double fb[9];
    const double rb = PL(a, R, PBRHO)[i0];
    for (int i = 0; i < 9; ++i) fb[i] = PL(a, R, PBF + i)[i0] + rb;
    double g[kTangents] = {0, 0, 0, 0};
    if (R.bc_x == 1 && x == R.nx - 1) {
        const double U = R.u_in;
        const int dirs[3] = {2, 6, 8};
        for (int m = 0; m < 3; ++m) {
            const int i = dirs[m];
            fb[i] += a.ain[adj_hist(R) + (size_t)m * R.ny + y];
            const double h = a.hist[m * R.ny + y];
            const double p = a.fs[(size_t)i * P + nid(R, R.nx - 1, wrap(y - cy_of(i), R.ny))];
            a.aout[adj_hist(R) + (size_t)m * R.ny + y] = fb[i] / (1.0 + U);
            const double dU = fb[i] * (p - h) / ((1.0 + U) * (1.0 + U));
            for (int t = 0; t < kTangents; ++t) g[t] += dU * R.t_u_in[t];
            fb[i] = U * fb[i] / (1.0 + U);   // adjoint of the pulled f*_i(nx-1, y - c_iy)
        }
    }
    if (R.bc_x == 1 && x == 0) {
        const double u = R.u_in;
        double f[9];
        for (int i = 0; i < 9; ++i) f[i] = PL(a, R, PF + i)[i0];
        const double rin = (f[0] + f[3] + f[4] + 2.0 * (f[2] + f[6] + f[8])) / (1.0 - u);
        const double rinb = fb[1] * (2.0 / 3.0) * u + (fb[5] + fb[7]) * u / 6.0;
        const double ub = fb[1] * (2.0 / 3.0) * rin + (fb[5] + fb[7]) * rin / 6.0 + rinb * rin / (1.0 - u);
        fb[2] += fb[1];
        fb[6] += fb[5];
        fb[8] += fb[7];
        fb[3] += 0.5 * (fb[7] - fb[5]);
        fb[4] += 0.5 * (fb[5] - fb[7]);
        const double q = rinb / (1.0 - u);
        fb[0] += q;
        fb[3] += q;
        fb[4] += q;
        fb[2] += 2.0 * q;
        fb[6] += 2.0 * q;
        fb[8] += 2.0 * q;
        fb[1] = fb[5] = fb[7] = 0.0;
        for (int t = 0; t < kTangents; ++t) g[t] += ub * R.t_u_in[t];
    }
    for (int i = 0; i < 9; ++i) PL(a, R, PBF + i)[i0] = fb[i];
    add_theta(PL(a, R, PTH), P, i0, g);
}

// transposed streaming (plain pulls, interpolated bounce-back, the convective outlet's pulls):
// lambda_f* and lambda_T of state n
__global__ __launch_bounds__(256) void kb_stream(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    int x, y;
    if (!node_kernel_index(R, x, y)) return;
    const size_t P = plane_of(R), i0 = nid(R, x, y);
    a.aout[adj_T(R) + i0] = PL(a, R, PBT)[i0];
    if (solid_at(R, x, y)) {
        for (int j = 0; j < 9; ++j) a.aout[(size_t)j * P + i0] = 0.0;
        return;
    }
    const int bw = 2 * R.cyl_r + 3;
    const bool near_y = near_cylinder(R, x, y);
    auto qv = [&](int qx, int qy, int i) {
        return ((const double *)R.qtab)[((qy - (R.cyl_y - R.cyl_r - 1)) * bw + (qx - (R.cyl_x - R.cyl_r - 1))) * 8 + (i - 1)];
    };
    const double *fb = PL(a, R, PBF);
    for (int j = 0; j < 9; ++j) {
        double l = 0.0;
        // plain pull of population j by x + c_j
        int px = x + cx_of(j);
        const int py = wrap(y + cy_of(j), R.ny);
        bool in = true;
        if (R.bc_x == 0) px = wrap(px, R.nx);
        else in = px >= 0 && px < R.nx;
        if (in && !solid_at(R, px, py)) {
            l += fb[(size_t)j * P + nid(R, px, py)];
            // interpolated bounce-back at x + c_j through its cut link opp(j): the neighbour term
            if (j > 0 && near_cylinder(R, px, py)) {
                const double v = qv(px, py, opp_of(j));
                if (v > 0.0 && v < 1.0) l += (1.0 - v) * fb[(size_t)opp_of(j) * P + nid(R, px, py)];
            }
        }
        // interpolated bounce-back of this node's own cut links
        if (j > 0 && near_y) {
            for (int i = 1; i < 9; ++i) {
                const double v = qv(x, y, i);
                if (v == 0.0) continue;
                const double b = fb[(size_t)i * P + i0];
                if (opp_of(i) == j) {
                    if (v > 2.0) l += b;
                    else if (v > 0.0) l += v * b;
                    else l += b / (-v);
                }
                if (i == j && v < 0.0) l += (-v - 1.0) / (-v) * b;
            }
        }
        // convective outlet: the last column's populations 2, 6, 8 take f*_j(nx-1, y') of row y' + c_jy
        if (R.bc_x == 1 && x == R.nx - 1 && (j == 2 || j == 6 || j == 8))
            l += fb[(size_t)j * P + nid(R, R.nx - 1, wrap(y + cy_of(j), R.ny))];
        a.aout[(size_t)j * P + i0] = l;
    }
}

// fixed-order tree sum of one value per thread of a 256-thread workgroup (the result in thread 0)
__device__ inline double tree_sum256(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

// the per-node parameter contributions summed over a block of rows per workgroup, in a fixed order
__global__ __launch_bounds__(256) void kb_theta_part(const RunDev *__restrict__ runs, int run, AdjArgs a)
{
    const RunDev &R = runs[run];
    __shared__ double red[256];
    const int nb = theta_blocks(R.ny);
    const int y0 = (int)((long long)blockIdx.x * R.ny / nb), y1 = (int)((long long)(blockIdx.x + 1) * R.ny / nb);
    double s[kTangents] = {0.0, 0.0, 0.0, 0.0};
    for (int y = y0; y < y1; ++y)
        for (int x = threadIdx.x; x < R.nx; x += 256) {
            const size_t i0 = nid(R, x, y);
#pragma unroll
            for (int t = 0; t < kTangents; ++t) s[t] += PL(a, R, PTH + t)[i0];
        }
    for (int t = 0; t < kTangents; ++t) {
        const double v = tree_sum256(s[t], red);
        if (threadIdx.x == 0) theta_parts(a, R)[(size_t)blockIdx.x * kTangents + t] = v;
    }
}

// the row blocks' sums in a fixed order (and the Nu sample's explicit part) onto the incoming
// accumulated gradient
__global__ __launch_bounds__(256) void kb_theta(const RunDev *__restrict__ runs, int run, AdjArgs a, int with_probe)
{
    const RunDev &R = runs[run];
    __shared__ double red[256];
    const int nb = theta_blocks(R.ny);
    for (int t = 0; t < kTangents; ++t) {
        const double v = (int)threadIdx.x < nb ? theta_parts(a, R)[(size_t)threadIdx.x * kTangents + t] : 0.0;
        const double sum = tree_sum256(v, red);
        if (threadIdx.x == 0) {
            double tot = a.ain[adj_theta(R) + t] + sum;
            if (with_probe) tot += probe_theta(a, R)[t];
            a.aout[adj_theta(R) + t] = tot;
        }
    }
}

// Contributions of the initial state to the gradient (appended to the accumulated one in place):
// solid nodes hold T_w (the superheat); a default state, f* = f^eq(rho_l, (u_in, 0)) with the same
// outlet history, depends on u_in.  One workgroup, fixed order.
__global__ __launch_bounds__(256) void kb_initial(const RunDev *__restrict__ runs, int run, double *adj, int default_state)
{
    const RunDev &R = runs[run];
    __shared__ double red[256];
    const size_t P = plane_of(R);
    double s[kTangents] = {0, 0, 0, 0};
    Dual feq[9];
    const bool inlet = R.bc_x == 1;
    if (default_state && inlet) equilibrium<Dual>(Dual(R.rho_l), seed(R.u_in, 0), Dual(0.0), feq);
    for (long long k = threadIdx.x; k < (long long)R.nx * R.ny; k += 256) {
        const int x = (int)(k % R.nx), y = (int)(k / R.nx);
        const size_t i0 = nid(R, x, y);
        if (solid_at(R, x, y)) {
            for (int t = 0; t < kTangents; ++t) s[t] += adj[adj_T(R) + i0] * R.t_T_w[t];
            continue;
        }
        if (default_state && inlet) {
            double du = 0.0;
            for (int i = 0; i < 9; ++i) du += adj[(size_t)i * P + i0] * feq[i].d[0];
            if (x == R.nx - 1) {
                const int dirs[3] = {2, 6, 8};
                for (int m = 0; m < 3; ++m) du += adj[adj_hist(R) + (size_t)m * R.ny + y] * feq[dirs[m]].d[0];
            }
            for (int t = 0; t < kTangents; ++t) s[t] += du * R.t_u_in[t];
        }
    }
    for (int t = 0; t < kTangents; ++t) {
        red[threadIdx.x] = s[t];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) adj[adj_theta(R) + t] += red[0];
        __syncthreads();
    }
}

}  // namespace

size_t adjoint_scratch_doubles(int nx, int ny, int pitch)
{
    (void)nx;
    return (size_t)NPLANES * ny * pitch + 2 * kMaxProbes + kTangents + (size_t)kThetaBlocks * kTangents;
}

size_t adjoint_state_doubles(int nx, int ny, int pitch)
{
    (void)nx;
    return 10 * (size_t)ny * pitch + 3 * (size_t)ny + kTangents;
}

hipError_t launch_adjoint_step(const RunDev *runs_dev, int run, const RunDev &Rh, const double *fs, const double *hist,
                               const double *T, const double *ain, double *aout, double *scratch, long long step,
                               double nu_weight, hipStream_t st)
{
    const bool fon = step >= Rh.warmup;
    const bool thermal = fon && Rh.rk > 0;
    AdjArgs a{fs, hist, T, ain, aout, scratch, step, nu_weight, 0, fon ? 1 : 0, thermal ? 1 : 0};
    const long long n = (long long)Rh.nx * Rh.ny;
    const int grid = (int)((n + 255) / 256);
    auto go = [&](void (*k)(const RunDev *, int, AdjArgs), int stage) {
        a.stage = stage;
        hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, st, runs_dev, run, a);
    };
    // forward recompute
    go(ka_stream, 0);
    if (fon) go(ka_psi, 0);
    go(ka_force, 0);
    if (thermal) {
        go(ka_frozen, 0);
        for (int s = 1; s < Rh.rk; ++s) go(ka_stage, s);
    }
    // reverse
    go(kb_init, 0);
    if (thermal) {
        for (int s = Rh.rk; s >= 1; --s) go(kb_stage, s);
        go(kb_coef, 0);
        go(kb_frozen_gather, 0);
    }
    const bool probe = fon && nu_weight != 0.0 && Rh.np > 0;
    if (probe) {
        hipLaunchKernelGGL(kb_probe, dim3(1), dim3(256), 0, st, runs_dev, run, a);
        go(kb_nu, 0);
    }
    go(kb_collide, 0);
    if (fon) go(kb_psi, 0);
    go(kb_bc, 0);
    go(kb_stream, 0);
    hipLaunchKernelGGL(kb_theta_part, dim3(theta_blocks(Rh.ny)), dim3(256), 0, st, runs_dev, run, a);
    hipLaunchKernelGGL(kb_theta, dim3(1), dim3(256), 0, st, runs_dev, run, a, probe ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_adjoint_initial(const RunDev *runs_dev, int run, double *adj, bool default_state, hipStream_t st)
{
    hipLaunchKernelGGL(kb_initial, dim3(1), dim3(256), 0, st, runs_dev, run, adj, default_state ? 1 : 0);
    return hipGetLastError();
}

}  // namespace lbm
