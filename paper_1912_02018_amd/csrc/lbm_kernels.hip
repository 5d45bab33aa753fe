// gfx950 kernels of one coupled step of the central-moment pseudopotential LBM with a
// finite-difference temperature equation (Saito et al., arXiv:1912.02018, Sec. II and IV A).
//
// Data layout in HBM (per run): populations in structure-of-arrays planes [9][ny][pitch]
// (x fastest, 64-element aligned rows) so that a wavefront reads 64 consecutive nodes of one
// population; temperature, density and velocity planes [ny][pitch] in the compute type.
//
// Kernels
//   k_lbm      streaming (pull) with the boundary conditions, density/momentum, psi of the EOS on
//              an LDS tile with a 2-node halo, 24-neighbour interaction force, gravity, and the
//              central-moment collision reconstructed in closed form f* = M^-1 N(-u) k*.
//              Writes f*, rho, u and the outlet history.  Bandwidth bound.
//   k_thermal  all Runge-Kutta stages of the temperature equation for one tile in LDS, the tile
//              carrying a halo of 2 nodes per stage so the stages never leave the CU.
//   k_diag_*   FP64 mass and wall heat-flux reductions in a fixed order (bitwise reproducible).
//   k_init     f* := f^eq(rho, u), outlet history, temperature from host-provided fields.
// No MFMA: every kernel is a stencil or an elementwise map.

#include "lbm_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <type_traits>

namespace lbm {
namespace {

// ------------------------------------------------------------------------------------------
// Lattice (eq. velVec) and interaction-stencil weights (eq. interForce)
// ------------------------------------------------------------------------------------------
__host__ __device__ constexpr int cx_of(int i) { return i == 1 || i == 5 || i == 7 ? 1 : (i == 2 || i == 6 || i == 8 ? -1 : 0); }
__host__ __device__ constexpr int cy_of(int i) { return i == 3 || i == 5 || i == 8 ? 1 : (i == 4 || i == 6 || i == 7 ? -1 : 0); }
__host__ __device__ constexpr int opp_of(int i) { return i == 0 ? 0 : (i % 2 == 1 ? i + 1 : i - 1); }
__host__ __device__ constexpr double lat_w(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }
__host__ __device__ constexpr double st_w(int e2)
{
    return e2 == 1 ? 4.0 / 21.0 : e2 == 2 ? 4.0 / 45.0 : e2 == 4 ? 1.0 / 60.0 : e2 == 5 ? 2.0 / 315.0 : e2 == 8 ? 1.0 / 5040.0 : 0.0;
}

// ------------------------------------------------------------------------------------------
// Storage <-> compute conversion.  Reduced-precision storage holds f_i - w_i rho_ref.
// ------------------------------------------------------------------------------------------
template <typename S> struct Conv;
template <> struct Conv<double> {
    __device__ static double ld(double v, double) { return v; }
    __device__ static double st(double v, double) { return v; }
};
template <> struct Conv<float> {
    __device__ static float ld(float v, float) { return v; }
    __device__ static float st(float v, float) { return v; }
};
template <> struct Conv<__half> {
    __device__ static float ld(__half v, float s) { return __half2float(v) + s; }
    __device__ static __half st(float v, float s) { return __float2half_rn(v - s); }
};
template <> struct Conv<__hip_bfloat16> {
    __device__ static float ld(__hip_bfloat16 v, float s) { return __bfloat162float(v) + s; }
    __device__ static __hip_bfloat16 st(float v, float s) { return __float2bfloat16(v - s); }
};

template <typename S> using CT = typename std::conditional<std::is_same<S, double>::value, double, float>::type;

__device__ inline int wrap_small(int a, int n)
{
    // a in [-n, 2n)
    return a < 0 ? a + n : (a >= n ? a - n : a);
}

__device__ inline int wrap_any(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

__device__ inline bool solid_at(const RunDev &R, int x, int y)
{
    if (R.cyl_r <= 0) return false;
    int dx = x - R.cyl_x, dy = y - R.cyl_y;
    return dx * dx + dy * dy <= R.cyl_r * R.cyl_r;
}

// Position kinds of the extended field: a node of the domain, an inlet ghost column (x < 0,
// rho/u of column 0, T = T_sat) or an outlet ghost column (x >= nx, copy of column nx-1).
enum { NODE = 0, INLET_GHOST = 1, OUTLET_GHOST = 2 };

// Map a lattice position to the domain node whose values it carries.
__device__ inline int map_pos(const RunDev &R, int gx, int gy, int &rx, int &ry)
{
    ry = wrap_any(gy, R.ny);
    if (R.bc_x == 0) {
        rx = wrap_any(gx, R.nx);
        return NODE;
    }
    if (gx < 0) { rx = 0; return INLET_GHOST; }
    if (gx >= R.nx) { rx = R.nx - 1; return OUTLET_GHOST; }
    rx = gx;
    return NODE;
}

// ------------------------------------------------------------------------------------------
// Run constants in the compute type
// ------------------------------------------------------------------------------------------
template <typename C> struct Consts {
    C omega, sigma, G, gx, gy, rho_gref, rho_w, T_sat, T_w, Tc, kappa, a, b, Rg, u_in, alpha, cv;
    C shiftw[9];
    __device__ explicit Consts(const RunDev &R)
    {
        omega = (C)R.omega; sigma = (C)R.sigma; G = (C)R.G; gx = (C)R.gx; gy = (C)R.gy;
        rho_gref = (C)R.rho_gref; rho_w = (C)R.rho_w; T_sat = (C)R.T_sat; T_w = (C)R.T_w;
        Tc = (C)R.Tc; kappa = (C)R.kappa; a = (C)R.eos_a; b = (C)R.eos_b; Rg = (C)R.eos_R;
        u_in = (C)R.u_in; alpha = (C)R.alpha; cv = (C)R.cv;
#pragma unroll
        for (int i = 0; i < 9; ++i) shiftw[i] = (C)(lat_w(i) * R.shift);
    }
};

// Peng-Robinson pressure (eq. eos) and the EOS-consistent pseudopotential (eq. potential).
template <typename C> __device__ inline C pr_pressure(const Consts<C> &K, C rho, C T)
{
    C s = (C)1 + K.kappa * ((C)1 - sqrt(T / K.Tc));
    C phi = s * s;
    return rho * K.Rg * T / ((C)1 - K.b * rho) - K.a * phi * rho * rho / ((C)1 + (C)2 * K.b * rho - K.b * K.b * rho * rho);
}

template <typename C> __device__ inline C pseudopotential(const Consts<C> &K, C rho, C T)
{
    const C cs2 = (C)(1.0 / 3.0);
    C p = pr_pressure(K, rho, T);
    return sqrt((C)2 * (p - rho * cs2) / (K.G * cs2));
}

// ------------------------------------------------------------------------------------------
// Streaming of one fluid node: f_i(x) = f*_i(x - c_i) with the boundary conditions
// ------------------------------------------------------------------------------------------
template <typename S, typename C>
__device__ inline C ldf(const S *__restrict__ f, size_t plane, int pitch, int i, int x, int y, const Consts<C> &K)
{
    return Conv<S>::ld(f[(size_t)i * plane + (size_t)y * pitch + x], K.shiftw[i]);
}

__device__ inline double link_q(const RunDev &R, int x, int y, int i)
{
    // smaller root of |d - q c|^2 = R^2, d = node - centre (exact integers up to the sqrt)
    double dx = x - R.cyl_x, dy = y - R.cyl_y, cx = cx_of(i), cy = cy_of(i);
    double c2 = cx * cx + cy * cy, dc = dx * cx + dy * cy;
    double Rr = R.cyl_r;
    double disc = dc * dc - c2 * (dx * dx + dy * dy - Rr * Rr);
    return (dc - sqrt(disc)) / c2;
}

template <typename S, typename C>
__device__ void stream_node(const RunDev &R, const Consts<C> &K, const S *__restrict__ fin,
                            const C *__restrict__ hin, int x, int y, C f[9])
{
    const int nx = R.nx, ny = R.ny, P = R.pitch;
    const size_t plane = (size_t)ny * P;
    const bool periodic = R.bc_x == 0;
    const int ym = y == 0 ? ny - 1 : y - 1;
    const int yp = y == ny - 1 ? 0 : y + 1;
    const int xm = periodic ? (x == 0 ? nx - 1 : x - 1) : x - 1;
    const int xp = periodic ? (x == nx - 1 ? 0 : x + 1) : x + 1;
    const bool near = R.cyl_r > 0 && abs(x - R.cyl_x) <= R.cyl_r + 1 && abs(y - R.cyl_y) <= R.cyl_r + 1;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int xs = cx_of(i) > 0 ? xm : (cx_of(i) < 0 ? xp : x);
        const int ys = cy_of(i) > 0 ? ym : (cy_of(i) < 0 ? yp : y);
        if (!periodic && (xs < 0 || xs >= nx)) { f[i] = (C)0; continue; }
        if (near && solid_at(R, xs, ys)) {
            // linear interpolated bounce-back on the curved wall
            const int o = opp_of(i);
            const double q = link_q(R, x, y, i);
            const C fo = ldf<S, C>(fin, plane, P, o, x, y, K);
            if (q < 0.5) {
                int xn = x + cx_of(i), yn = wrap_small(y + cy_of(i), ny);
                if (periodic) xn = wrap_small(xn, nx);
                const bool fluid_n = xn >= 0 && xn < nx && !solid_at(R, xn, yn);
                if (fluid_n) {
                    const C q2 = (C)(2.0 * q);
                    f[i] = q2 * fo + ((C)1 - q2) * ldf<S, C>(fin, plane, P, o, xn, yn, K);
                } else {
                    f[i] = fo;
                }
            } else {
                const C q2 = (C)(2.0 * q);
                f[i] = fo / q2 + (q2 - (C)1) / q2 * ldf<S, C>(fin, plane, P, i, x, y, K);
            }
        } else {
            f[i] = ldf<S, C>(fin, plane, P, i, xs, ys, K);
        }
    }
    if (!periodic) {
        if (x == nx - 1) {
            // convective outflow: f^{n+1}(N) = (f^n(N) + U f^{n+1}(N-1)) / (1 + U), i in {2,6,8}
            const C U = K.u_in;
            const C p2 = ldf<S, C>(fin, plane, P, 2, nx - 1, y, K);
            const C p6 = ldf<S, C>(fin, plane, P, 6, nx - 1, yp, K);
            const C p8 = ldf<S, C>(fin, plane, P, 8, nx - 1, ym, K);
            f[2] = (hin[0 * ny + y] + U * p2) / ((C)1 + U);
            f[6] = (hin[1 * ny + y] + U * p6) / ((C)1 + U);
            f[8] = (hin[2 * ny + y] + U * p8) / ((C)1 + U);
        }
        if (x == 0) {
            // velocity inlet (u_in, 0): unknowns 1, 5, 7
            const C u = K.u_in;
            const C rin = (f[0] + f[3] + f[4] + (C)2 * (f[2] + f[6] + f[8])) / ((C)1 - u);
            f[1] = f[2] + (C)(2.0 / 3.0) * rin * u;
            f[5] = f[6] - (C)0.5 * (f[3] - f[4]) + rin * u / (C)6;
            f[7] = f[8] + (C)0.5 * (f[3] - f[4]) + rin * u / (C)6;
        }
    }
}

// ------------------------------------------------------------------------------------------
// k_lbm: streaming + moments + psi + force + central-moment collision
// ------------------------------------------------------------------------------------------
template <typename S, int TX, int TY, bool WRITE_F>
__global__ __launch_bounds__(256) void k_lbm(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles,
                                             int pf, int pt, int ph, long long step)
{
    using C = CT<S>;
    constexpr int H = 2;
    constexpr int RW = TX + 2 * H, RH = TY + 2 * H, RN = RW * RH, TN = TX * TY;
    __shared__ C s_psi[RN];
    __shared__ C s_m[5][TN];  // rho, jx, jy, sum f (cx^2 - cy^2), sum f cx cy

    const Tile t = tiles[blockIdx.x];
    const RunDev &R = runs[t.run];
    const Consts<C> K(R);
    const int x0 = t.tx * TX, y0 = t.ty * TY;
    const int nx = R.nx, ny = R.ny, P = R.pitch;
    const bool fon = step >= R.warmup;
    const S *__restrict__ fin = (const S *)R.f[pf];
    S *__restrict__ fout = (S *)R.f[pf ^ 1];
    const C *__restrict__ Tc = (const C *)R.T[pt];
    const C *__restrict__ hin = (const C *)R.hist[ph];
    C *__restrict__ hout = (C *)R.hist[ph ^ 1];

    // phase 1: density (and psi) on the tile plus halo, raw moments on the tile
    for (int p = threadIdx.x; p < RN; p += blockDim.x) {
        const int lx = p % RW, ly = p / RW;
        const int gx = x0 - H + lx, gy = y0 - H + ly;
        const bool own = lx >= H && lx < H + TX && ly >= H && ly < H + TY && gx < nx && gy < ny;
        if (!fon && !own) continue;
        int rx, ry;
        const int kind = map_pos(R, gx, gy, rx, ry);
        C rho, T;
        if (solid_at(R, rx, ry)) {
            rho = K.rho_w;
            T = K.T_w;
            if (own) {
                const int q = (ly - H) * TX + (lx - H);
                s_m[0][q] = rho; s_m[1][q] = 0; s_m[2][q] = 0; s_m[3][q] = 0; s_m[4][q] = 0;
            }
        } else {
            C f[9];
            stream_node<S, C>(R, K, fin, hin, rx, ry, f);
            rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
            T = kind == INLET_GHOST ? K.T_sat : Tc[(size_t)ry * P + rx];
            if (own) {
                const int q = (ly - H) * TX + (lx - H);
                s_m[0][q] = rho;
                s_m[1][q] = (f[1] - f[2]) + (f[5] - f[6]) + (f[7] - f[8]);
                s_m[2][q] = (f[3] - f[4]) + (f[5] - f[6]) + (f[8] - f[7]);
                s_m[3][q] = (f[1] + f[2]) - (f[3] + f[4]);
                s_m[4][q] = (f[5] + f[6]) - (f[7] + f[8]);
                if (WRITE_F && R.bc_x == 1 && gx == nx - 1) {
                    hout[0 * ny + gy] = f[2];
                    hout[1 * ny + gy] = f[6];
                    hout[2 * ny + gy] = f[8];
                }
            }
        }
        if (fon) s_psi[p] = pseudopotential(K, rho, T);
    }
    __syncthreads();

    C *__restrict__ orho = (C *)R.rho;
    C *__restrict__ oux = (C *)R.ux;
    C *__restrict__ ouy = (C *)R.uy;
    const size_t plane = (size_t)ny * P;
    const C cs2 = (C)(1.0 / 3.0);

    // phase 2: force, velocity, collision of the tile nodes
    for (int q = threadIdx.x; q < TN; q += blockDim.x) {
        const int lx = q % TX, ly = q / TX;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= nx || gy >= ny) continue;
        const size_t idx = (size_t)gy * P + gx;
        if (solid_at(R, gx, gy)) {
            orho[idx] = K.rho_w;
            oux[idx] = 0;
            ouy[idx] = 0;
            continue;
        }
        const C rho = s_m[0][q], jx = s_m[1][q], jy = s_m[2][q], m4 = s_m[3][q], m5 = s_m[4][q];
        C Fx = 0, Fy = 0, A = 0;
        if (fon) {
            const int c = (ly + H) * RW + (lx + H);
            C sx = 0, sy = 0;
#pragma unroll
            for (int ey = -2; ey <= 2; ++ey)
#pragma unroll
                for (int ex = -2; ex <= 2; ++ex) {
                    if (ex == 0 && ey == 0) continue;
                    const C w = (C)st_w(ex * ex + ey * ey);
                    const C ps = s_psi[c + ey * RW + ex];
                    sx += w * ps * (C)ex;
                    sy += w * ps * (C)ey;
                }
            const C psi0 = s_psi[c];
            const C Fmx = -K.G * cs2 * psi0 * sx;
            const C Fmy = -K.G * cs2 * psi0 * sy;
            A = (C)2 * K.sigma * (Fmx * Fmx + Fmy * Fmy) / (psi0 * psi0);
            Fx = Fmx + (rho - K.rho_gref) * K.gx;
            Fy = Fmy + (rho - K.rho_gref) * K.gy;
        }
        const C U = (jx + (C)0.5 * Fx) / rho;
        const C V = (jy + (C)0.5 * Fy) / rho;
        orho[idx] = rho;
        oux[idx] = U;
        ouy[idx] = V;
        if (!WRITE_F) continue;

        // pre-collision central moments k4, k5 from raw moments (rows 4, 5 of N(u))
        const C k4 = (U * U - V * V) * rho - (C)2 * U * jx + (C)2 * V * jy + m4;
        const C k5 = U * V * rho - V * jx - U * jy + m5;
        // post-collision central moments (eq. postColl2)
        const C k0 = rho, k1 = (C)0.5 * Fx, k2 = (C)0.5 * Fy;
        const C k3 = (C)(2.0 / 3.0) * rho + A;
        const C k4s = ((C)1 - K.omega) * k4, k5s = ((C)1 - K.omega) * k5;
        const C k6 = Fy / (C)6, k7 = Fx / (C)6;
        const C k8 = rho / (C)9 + A / (C)3;
        // raw moments m* = N(-u) k*
        const C UU = U * U, VV = V * V, UV = U * V;
        const C r0 = k0;
        const C r1 = U * k0 + k1;
        const C r2 = V * k0 + k2;
        const C r3 = (UU + VV) * k0 + (C)2 * U * k1 + (C)2 * V * k2 + k3;
        const C r4 = (UU - VV) * k0 + (C)2 * U * k1 - (C)2 * V * k2 + k4s;
        const C r5 = UV * k0 + V * k1 + U * k2 + k5s;
        const C r6 = UU * V * k0 + (C)2 * UV * k1 + UU * k2 + (C)0.5 * V * (k3 + k4s) + (C)2 * U * k5s + k6;
        const C r7 = U * VV * k0 + VV * k1 + (C)2 * UV * k2 + (C)0.5 * U * (k3 - k4s) + (C)2 * V * k5s + k7;
        const C r8 = UU * VV * k0 + (C)2 * U * VV * k1 + (C)2 * UU * V * k2 + (C)0.5 * (UU + VV) * k3 -
                     (C)0.5 * (UU - VV) * k4s + (C)4 * UV * k5s + (C)2 * V * k6 + (C)2 * U * k7 + k8;
        // populations f* = M^-1 m*
        C fs[9];
        fs[0] = r0 - r3 + r8;
        fs[1] = (C)0.5 * (r1 - r7 - r8) + (C)0.25 * (r3 + r4);
        fs[2] = (C)0.5 * (-r1 + r7 - r8) + (C)0.25 * (r3 + r4);
        fs[3] = (C)0.5 * (r2 - r6 - r8) + (C)0.25 * (r3 - r4);
        fs[4] = (C)0.5 * (-r2 + r6 - r8) + (C)0.25 * (r3 - r4);
        fs[5] = (C)0.25 * (r5 + r6 + r7 + r8);
        fs[6] = (C)0.25 * (r5 - r6 - r7 + r8);
        fs[7] = (C)0.25 * (-r5 - r6 + r7 + r8);
        fs[8] = (C)0.25 * (-r5 + r6 - r7 + r8);
#pragma unroll
        for (int i = 0; i < 9; ++i) fout[(size_t)i * plane + idx] = Conv<S>::st(fs[i], K.shiftw[i]);
    }
}

// ------------------------------------------------------------------------------------------
// k_thermal: Runge-Kutta update of the temperature equation (eq. energy) on an LDS tile
// ------------------------------------------------------------------------------------------
template <typename C, int TX, int TY, int NS>
__global__ __launch_bounds__(256) void k_thermal(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles, int pt)
{
    constexpr int H = 2 * NS;  // frozen-field halo: 2 nodes per stage
    constexpr int RW = TX + 2 * H, RH = TY + 2 * H, RN = RW * RH, TN = TX * TY;
    constexpr int MAXPT = (RN + 255) / 256;
    __shared__ C s_ux[RN], s_uy[RN], s_T0[RN], s_Y[RN];  // s_Y holds rho until the invariants exist
    __shared__ C s_gx[RN], s_gy[RN], s_c1[RN], s_c2[RN];
    __shared__ C s_acc[TN];

    const Tile t = tiles[blockIdx.x];
    const RunDev &R = runs[t.run];
    const Consts<C> K(R);
    const int x0 = t.tx * TX, y0 = t.ty * TY;
    const int nx = R.nx, ny = R.ny, P = R.pitch;
    const C *__restrict__ Tin = (const C *)R.T[pt];
    C *__restrict__ Tout = (C *)R.T[pt ^ 1];
    const C *__restrict__ grho = (const C *)R.rho;
    const C *__restrict__ gux = (const C *)R.ux;
    const C *__restrict__ guy = (const C *)R.uy;

    // load the frozen fields and T^n on the whole region
    for (int p = threadIdx.x; p < RN; p += blockDim.x) {
        const int lx = p % RW, ly = p / RW;
        int rx, ry;
        const int kind = map_pos(R, x0 - H + lx, y0 - H + ly, rx, ry);
        const size_t idx = (size_t)ry * P + rx;
        s_Y[p] = grho[idx];
        s_ux[p] = gux[idx];
        s_uy[p] = guy[idx];
        s_T0[p] = kind == INLET_GHOST ? K.T_sat : Tin[idx];
    }
    for (int q = threadIdx.x; q < TN; q += blockDim.x) s_acc[q] = 0;
    __syncthreads();

    // stage-invariant coefficients on the region shrunk by 2:
    //   gx, gy = alpha grad(rho)/rho;  c1 = -div(u) R rho/(1 - b rho) / (rho cv);
    //   c2 = div(u) a rho^2/(1 + 2 b rho - b^2 rho^2) / (rho cv); source(T) = T (c1 + c2 phi'(T))
    for (int p = threadIdx.x; p < RN; p += blockDim.x) {
        const int lx = p % RW, ly = p / RW;
        if (lx < 2 || lx >= RW - 2 || ly < 2 || ly >= RH - 2) continue;
        C grx = 0, gry = 0, dv = 0;
#pragma unroll
        for (int ey = -2; ey <= 2; ++ey)
#pragma unroll
            for (int ex = -2; ex <= 2; ++ex) {
                if (ex == 0 && ey == 0) continue;
                const C w = (C)st_w(ex * ex + ey * ey);
                const int n = p + ey * RW + ex;
                grx += w * s_Y[n] * (C)ex;
                gry += w * s_Y[n] * (C)ey;
                dv += w * (s_ux[n] * (C)ex + s_uy[n] * (C)ey);
            }
        const C rho = s_Y[p];
        s_gx[p] = K.alpha * grx / rho;
        s_gy[p] = K.alpha * gry / rho;
        const C D = dv / (rho * K.cv);
        s_c1[p] = -D * (rho * K.Rg / ((C)1 - K.b * rho));
        s_c2[p] = D * (K.a * rho * rho / ((C)1 + (C)2 * K.b * rho - K.b * K.b * rho * rho));
    }
    __syncthreads();
    for (int p = threadIdx.x; p < RN; p += blockDim.x) s_Y[p] = s_T0[p];
    __syncthreads();

    const C cd = R.upwind_kind == 1 ? (C)0.25 : (C)(1.0 / 12.0);
    for (int s = 1; s <= NS; ++s) {
        const int m = 2 * (NS - s);  // region of this stage: tile grown by m
        const int W = TX + 2 * m, Hh = TY + 2 * m, N = W * Hh;
        C kv[MAXPT];
#pragma unroll
        for (int j = 0; j < MAXPT; ++j) {
            kv[j] = 0;
            const int r = threadIdx.x + 256 * j;
            if (r >= N) continue;
            const int lx = H - m + r % W, ly = H - m + r / W;
            int rx, ry;
            const int kind = map_pos(R, x0 - H + lx, y0 - H + ly, rx, ry);
            if (kind == INLET_GHOST || solid_at(R, rx, ry)) continue;
            // an outlet ghost evaluates the operator at the last column of its row
            const int cx = kind == OUTLET_GHOST ? lx - (x0 - H + lx - (nx - 1)) : lx;
            const int c = ly * RW + cx;
            const C y0v = s_Y[c];
            const C u = s_ux[c], v = s_uy[c];
            const C xm2 = s_Y[c - 2], xm1 = s_Y[c - 1], xp1 = s_Y[c + 1], xp2 = s_Y[c + 2];
            const C ym2 = s_Y[c - 2 * RW], ym1 = s_Y[c - RW], yp1 = s_Y[c + RW], yp2 = s_Y[c + 2 * RW];
            const C conv = u * (-xp2 + (C)8 * xp1 - (C)8 * xm1 + xm2) / (C)12 + fabs(u) * cd * (xp2 - (C)4 * xp1 + (C)6 * y0v - (C)4 * xm1 + xm2) +
                           v * (-yp2 + (C)8 * yp1 - (C)8 * ym1 + ym2) / (C)12 + fabs(v) * cd * (yp2 - (C)4 * yp1 + (C)6 * y0v - (C)4 * ym1 + ym2);
            C gxT = 0, gyT = 0, lap = 0;
#pragma unroll
            for (int ey = -2; ey <= 2; ++ey)
#pragma unroll
                for (int ex = -2; ex <= 2; ++ex) {
                    if (ex == 0 && ey == 0) continue;
                    const C w = (C)st_w(ex * ex + ey * ey);
                    const C yn = s_Y[c + ey * RW + ex];
                    gxT += w * yn * (C)ex;
                    gyT += w * yn * (C)ey;
                    lap += (C)2 * w * (yn - y0v);
                }
            const C diff = K.alpha * lap + s_gx[c] * gxT + s_gy[c] * gyT;
            // phi'(T) = -kappa (1 + kappa (1 - sqrt(T/Tc))) / sqrt(T Tc)
            const C sq = sqrt(y0v / K.Tc);
            const C dphi = -K.kappa * ((C)1 + K.kappa * ((C)1 - sq)) / sqrt(y0v * K.Tc);
            const C src = y0v * (s_c1[c] + s_c2[c] * dphi);
            kv[j] = -conv + diff + src;
        }
        __syncthreads();  // every stage input has been read
#pragma unroll
        for (int j = 0; j < MAXPT; ++j) {
            const int r = threadIdx.x + 256 * j;
            if (r >= N) continue;
            const int lx = H - m + r % W, ly = H - m + r / W;
            const int c = ly * RW + lx;
            const bool in_tile = lx >= H && lx < H + TX && ly >= H && ly < H + TY;
            const int q = (ly - H) * TX + (lx - H);
            const C k = kv[j];
            if (NS == 4) {
                if (s == 1) { if (in_tile) s_acc[q] = k; s_Y[c] = s_T0[c] + (C)0.5 * k; }
                else if (s == 2) { if (in_tile) s_acc[q] += (C)2 * k; s_Y[c] = s_T0[c] + (C)0.5 * k; }
                else if (s == 3) { if (in_tile) s_acc[q] += (C)2 * k; s_Y[c] = s_T0[c] + k; }
                else { if (in_tile) s_acc[q] = s_T0[c] + (s_acc[q] + k) / (C)6; }
            } else {
                if (s == 1) { if (in_tile) s_acc[q] = k; s_Y[c] = s_T0[c] + k; }
                else { if (in_tile) s_acc[q] = s_T0[c] + (C)0.5 * (s_acc[q] + k); }
            }
        }
        __syncthreads();
    }

    for (int q = threadIdx.x; q < TN; q += blockDim.x) {
        const int gx = x0 + q % TX, gy = y0 + q / TX;
        if (gx >= nx || gy >= ny) continue;
        Tout[(size_t)gy * P + gx] = solid_at(R, gx, gy) ? K.T_w : s_acc[q];
    }
}

// ------------------------------------------------------------------------------------------
// Diagnostics: FP64 mass and wall heat flux, fixed reduction order
// ------------------------------------------------------------------------------------------
template <typename C>
__global__ __launch_bounds__(256) void k_diag_partial(const RunDev *__restrict__ runs, int run)
{
    const RunDev &R = runs[run];
    const C *__restrict__ rho = (const C *)R.rho;
    __shared__ double red[256];
    double s = 0.0;
    const long long n = (long long)R.nx * R.ny;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int x = (int)(k % R.nx), y = (int)(k / R.nx);
        if (!solid_at(R, x, y)) s += (double)rho[(size_t)y * R.pitch + x];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) R.partials[blockIdx.x] = red[0];
}

template <typename C>
__global__ __launch_bounds__(256) void k_diag_final(const RunDev *__restrict__ runs, int run, int pt, int accumulate)
{
    const RunDev &R = runs[run];
    const C *__restrict__ rho = (const C *)R.rho;
    const C *__restrict__ T = (const C *)R.T[pt];
    __shared__ double qp[kMaxProbes];
    for (int k = threadIdx.x; k < R.np; k += 256) {
        const double px = R.probes[2 * k], py = R.probes[2 * k + 1];
        const int x0 = (int)floor(px), y0 = (int)floor(py);
        const double fx = px - x0, fy = py - y0;
        const size_t i00 = (size_t)y0 * R.pitch + x0, i01 = i00 + R.pitch;
        const double r = (1 - fx) * (1 - fy) * (double)rho[i00] + fx * (1 - fy) * (double)rho[i00 + 1] +
                         (1 - fx) * fy * (double)rho[i01] + fx * fy * (double)rho[i01 + 1];
        const double tp = (1 - fx) * (1 - fy) * (double)T[i00] + fx * (1 - fy) * (double)T[i00 + 1] +
                          (1 - fx) * fy * (double)T[i01] + fx * fy * (double)T[i01 + 1];
        qp[k] = r * R.cv * R.alpha * (R.T_w - tp) / 1.5;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mass = 0.0;
        for (int b = 0; b < kDiagBlocks; ++b) mass += R.partials[b];
        double q = 0.0;
        for (int k = 0; k < R.np; ++k) q += qp[k];
        q = R.np > 0 ? q / R.np : 0.0;
        const double dT = R.T_w - R.T_sat;
        const double nu = (R.np > 0 && dT != 0.0) ? q * 2.0 * R.cyl_r / (R.rho_v * R.cv * R.alpha * dT) : 0.0;
        R.acc[0] = mass;
        R.acc[1] = q;
        R.acc[2] = nu;
        if (accumulate) {
            R.acc[3] += nu;
            R.acc[4] += 1.0;
        }
        if (!(mass == mass) || mass - mass != 0.0) R.acc[5] = 1.0;
    }
}

// ------------------------------------------------------------------------------------------
// Initial state: f* = f^eq(rho, u) (full Hermite, eq. equi), outlet history, temperature
// ------------------------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(256) void k_init(const RunDev *__restrict__ runs, int run)
{
    using C = CT<S>;
    const RunDev &R = runs[run];
    const Consts<C> K(R);
    // host-provided fields were uploaded into rho, ux, uy and T[0]
    const C *rho = (const C *)R.rho, *ux = (const C *)R.ux, *uy = (const C *)R.uy;
    C *T = (C *)R.T[0];
    S *f = (S *)R.f[0];
    C *hist = (C *)R.hist[0];
    const size_t plane = (size_t)R.ny * R.pitch;
    const long long n = (long long)R.nx * R.ny;
    const C cs2 = (C)(1.0 / 3.0);
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int x = (int)(k % R.nx), y = (int)(k / R.nx);
        const size_t idx = (size_t)y * R.pitch + x;
        const C r = rho[idx], u = ux[idx], v = uy[idx];
        C feq[9];
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
            f[(size_t)i * plane + idx] = Conv<S>::st(feq[i], K.shiftw[i]);
        }
        if (x == R.nx - 1) {
            hist[0 * R.ny + y] = feq[2];
            hist[1 * R.ny + y] = feq[6];
            hist[2 * R.ny + y] = feq[8];
        }
        if (solid_at(R, x, y)) T[idx] = K.T_w;
    }
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------
TileShape tile_shape(int precision, int rk)
{
    (void)rk;
    if (precision == 0) return TileShape{32, 16, 16, 16};
    return TileShape{32, 16, 32, 32};
}

template <typename S>
static hipError_t lbm_impl(bool write_f, const RunDev *runs, const Tile *tiles, int n, int pf, int pt, int ph,
                           long long step, hipStream_t st, int tx, int ty)
{
    if (n <= 0) return hipSuccess;
    if (tx == 32 && ty == 16) {
        if (write_f) k_lbm<S, 32, 16, true><<<n, 256, 0, st>>>(runs, tiles, pf, pt, ph, step);
        else k_lbm<S, 32, 16, false><<<n, 256, 0, st>>>(runs, tiles, pf, pt, ph, step);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lbm(int precision, bool write_f, const RunDev *runs_dev, const Tile *tiles, int n_tiles, int pf,
                      int pt, int ph, long long step, hipStream_t stream)
{
    const TileShape ts = tile_shape(precision, 4);
    switch (precision) {
    case 0: return lbm_impl<double>(write_f, runs_dev, tiles, n_tiles, pf, pt, ph, step, stream, ts.lbm_tx, ts.lbm_ty);
    case 1: return lbm_impl<float>(write_f, runs_dev, tiles, n_tiles, pf, pt, ph, step, stream, ts.lbm_tx, ts.lbm_ty);
    case 2: return lbm_impl<__half>(write_f, runs_dev, tiles, n_tiles, pf, pt, ph, step, stream, ts.lbm_tx, ts.lbm_ty);
    case 3: return lbm_impl<__hip_bfloat16>(write_f, runs_dev, tiles, n_tiles, pf, pt, ph, step, stream, ts.lbm_tx, ts.lbm_ty);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_thermal(int precision, int rk, const RunDev *runs_dev, const Tile *tiles, int n_tiles, int pt,
                          long long step, hipStream_t stream)
{
    (void)step;
    if (n_tiles <= 0) return hipSuccess;
    if (precision == 0) {
        if (rk == 4) k_thermal<double, 16, 16, 4><<<n_tiles, 256, 0, stream>>>(runs_dev, tiles, pt);
        else if (rk == 2) k_thermal<double, 16, 16, 2><<<n_tiles, 256, 0, stream>>>(runs_dev, tiles, pt);
        else return hipErrorInvalidValue;
    } else {
        if (rk == 4) k_thermal<float, 32, 32, 4><<<n_tiles, 256, 0, stream>>>(runs_dev, tiles, pt);
        else if (rk == 2) k_thermal<float, 32, 32, 2><<<n_tiles, 256, 0, stream>>>(runs_dev, tiles, pt);
        else return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_diag(int precision, const RunDev *runs_dev, int run, const RunDev &host_run, int pt, int accumulate,
                       hipStream_t stream)
{
    (void)host_run;
    if (precision == 0) {
        k_diag_partial<double><<<kDiagBlocks, 256, 0, stream>>>(runs_dev, run);
        k_diag_final<double><<<1, 256, 0, stream>>>(runs_dev, run, pt, accumulate);
    } else {
        k_diag_partial<float><<<kDiagBlocks, 256, 0, stream>>>(runs_dev, run);
        k_diag_final<float><<<1, 256, 0, stream>>>(runs_dev, run, pt, accumulate);
    }
    return hipGetLastError();
}

hipError_t launch_init(int precision, const RunDev *runs_dev, int run, const RunDev &host_run, hipStream_t stream)
{
    const long long n = (long long)host_run.nx * host_run.ny;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    switch (precision) {
    case 0: k_init<double><<<blocks, 256, 0, stream>>>(runs_dev, run); break;
    case 1: k_init<float><<<blocks, 256, 0, stream>>>(runs_dev, run); break;
    case 2: k_init<__half><<<blocks, 256, 0, stream>>>(runs_dev, run); break;
    case 3: k_init<__hip_bfloat16><<<blocks, 256, 0, stream>>>(runs_dev, run); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
