// Device code shared by the step kernels (lbm_kernels.hip) and the adjoint kernels
// (lbm_adjoint.hip): lattice and stencil constants, the arithmetic of the compute types (FP64, FP32,
// forward-mode tangents), storage conversions, the field extension at the domain edges, the run
// constants, the pseudopotential of the Peng-Robinson EOS and the central-moment collision of one node.
// Each translation unit that includes it gets its own internal copy.
#pragma once

#include "lbm_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <type_traits>

namespace lbm {
namespace {

// pointers into the workspace, in the global address space (global_load/store, not flat); class
// types (the tangent type) keep generic pointers, whose objects can be assigned
struct Dual;
template <typename T> struct GlobalPtr { using type = __attribute__((address_space(1))) T *; };
template <> struct GlobalPtr<Dual> { using type = Dual *; };
template <> struct GlobalPtr<const Dual> { using type = const Dual *; };
template <typename T> using gp = typename GlobalPtr<T>::type;
template <typename T> __device__ inline gp<const T> gin(const void *p) { return (gp<const T>)p; }
template <typename T> __device__ inline gp<T> gout(void *p) { return (gp<T>)p; }
// element e of a workspace array, addressed with a 32-bit byte offset from a uniform base
template <typename T> __device__ inline gp<T> at(void *base, unsigned e)
{
    return (gp<T>)((char *)base + e * (unsigned)sizeof(T));
}
template <typename T> __device__ inline T ld_at(const void *base, unsigned e)
{
    return *(gp<const T>)((const char *)base + e * (unsigned)sizeof(T));
}

// ------------------------------------------------------------------------------------------
// Lattice (eq. velVec) and interaction-stencil weights (eq. interForce)
// ------------------------------------------------------------------------------------------
__host__ __device__ constexpr int cx_of(int i) { return i == 1 || i == 5 || i == 7 ? 1 : (i == 2 || i == 6 || i == 8 ? -1 : 0); }
__host__ __device__ constexpr int cy_of(int i) { return i == 3 || i == 5 || i == 8 ? 1 : (i == 4 || i == 6 || i == 7 ? -1 : 0); }
__host__ __device__ constexpr int opp_of(int i) { return i == 0 ? 0 : (i % 2 == 1 ? i + 1 : i - 1); }
__host__ __device__ constexpr double lat_w(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }
constexpr double W1 = 4.0 / 21.0, W2 = 4.0 / 45.0, W4 = 1.0 / 60.0, W5 = 2.0 / 315.0, W8 = 1.0 / 5040.0;
constexpr double WSUM = 4.0 * W1 + 4.0 * W2 + 4.0 * W4 + 8.0 * W5 + 4.0 * W8;

// ------------------------------------------------------------------------------------------
// Arithmetic of the compute type: IEEE division and square root in FP64; the native gfx950
// reciprocal / square-root instructions (about 1 ulp) in FP32.
// ------------------------------------------------------------------------------------------
template <typename C> struct Ar;
template <> struct Ar<double> {
    __device__ static double rcp(double x) { return 1.0 / x; }
    __device__ static double sqrt_(double x) { return sqrt(x); }
};
template <> struct Ar<float> {
    __device__ static float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
};

// ------------------------------------------------------------------------------------------
// Forward-mode tangents: an FP64 value with kTangents directional derivatives.  Instantiating
// the step with this compute (and storage) type carries d(state)/d(parameter) for every
// parameter direction through exactly the arithmetic of the FP64 step (the value part is that
// step's value); comparisons and branches look at the value only.
// ------------------------------------------------------------------------------------------
struct Dual {
    double v, d[kTangents];
    Dual() = default;
    __host__ __device__ constexpr Dual(double x) : v(x), d{} {}
    __device__ explicit operator double() const { return v; }
};
__device__ inline Dual operator+(const Dual &a, const Dual &b)
{
    Dual r; r.v = a.v + b.v;
#pragma unroll
    for (int k = 0; k < kTangents; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
__device__ inline Dual operator-(const Dual &a, const Dual &b)
{
    Dual r; r.v = a.v - b.v;
#pragma unroll
    for (int k = 0; k < kTangents; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
__device__ inline Dual operator-(const Dual &a)
{
    Dual r; r.v = -a.v;
#pragma unroll
    for (int k = 0; k < kTangents; ++k) r.d[k] = -a.d[k];
    return r;
}
__device__ inline Dual operator*(const Dual &a, const Dual &b)
{
    Dual r; r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < kTangents; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
__device__ inline Dual operator/(const Dual &a, const Dual &b)
{
    Dual r; r.v = a.v / b.v;
    const double ib = 1.0 / b.v;
#pragma unroll
    for (int k = 0; k < kTangents; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
    return r;
}
__device__ inline Dual &operator+=(Dual &a, const Dual &b) { return a = a + b; }
__device__ inline bool operator==(const Dual &a, const Dual &b) { return a.v == b.v; }
__device__ inline bool operator<(const Dual &a, const Dual &b) { return a.v < b.v; }
__device__ inline bool operator>(const Dual &a, const Dual &b) { return a.v > b.v; }
template <> struct Ar<Dual> {
    __device__ static Dual rcp(const Dual &x)
    {
        Dual r; r.v = 1.0 / x.v;
#pragma unroll
        for (int k = 0; k < kTangents; ++k) r.d[k] = -x.d[k] * r.v * r.v;
        return r;
    }
    __device__ static Dual sqrt_(const Dual &x)
    {
        Dual r; r.v = sqrt(x.v);
        const double h = 0.5 / r.v;
#pragma unroll
        for (int k = 0; k < kTangents; ++k) r.d[k] = x.d[k] * h;
        return r;
    }
};

// ------------------------------------------------------------------------------------------
// Storage type S, its raw bit type in memory, and the conversion to the compute type;
// reduced-precision storage holds f_i - w_i rho_ref.
template <typename S> struct Conv;
template <> struct Conv<double> {
    using raw = double;
    __device__ static double ld(double v, double) { return v; }
    __device__ static double st(double v, double) { return v; }
};
template <> struct Conv<float> {
    using raw = float;
    __device__ static float ld(float v, float) { return v; }
    __device__ static float st(float v, float) { return v; }
};
// (the shift is added and subtracted as separate roundings, never fused with the product that
// produced the value: every kernel then stores and loads the same bits)
template <> struct Conv<__half> {
    using raw = unsigned short;
    __device__ static float ld(unsigned short v, float s)
    {
#pragma clang fp contract(off)
        return __half2float(__ushort_as_half(v)) + s;
    }
    __device__ static unsigned short st(float v, float s)
    {
#pragma clang fp contract(off)
        return __half_as_ushort(__float2half_rn(v - s));
    }
};
template <> struct Conv<Dual> {
    using raw = Dual;
    __device__ static Dual ld(const Dual &v, const Dual &) { return v; }
    __device__ static Dual st(const Dual &v, const Dual &) { return v; }
};
template <> struct Conv<__hip_bfloat16> {
    using raw = unsigned short;
    __device__ static float ld(unsigned short v, float s)
    {
#pragma clang fp contract(off)
        return __uint_as_float((unsigned)v << 16) + s;
    }
    __device__ static unsigned short st(float v, float s)
    {
#pragma clang fp contract(off)
        return __bfloat16_as_ushort(__float2bfloat16(v - s));
    }
};
template <typename S> using RawT = typename Conv<S>::raw;

// compute type of a storage type: FP64 and tangents compute in themselves, the rest in FP32
template <typename S>
using CT = typename std::conditional<std::is_same<S, double>::value || std::is_same<S, Dual>::value, S, float>::type;
template <typename C> constexpr bool is_dual = std::is_same<C, Dual>::value;

// |x| of the compute type (the tangent of |x| takes the sign of the value)
template <typename C> __device__ inline C absval(const C &x) { return fabs(x); }
template <> __device__ inline Dual absval<Dual>(const Dual &x) { return x.v < 0.0 ? -x : x; }

// a run constant in the compute type; tangent types take its derivatives along the parameter
// directions from the run description
template <typename C> __device__ inline C seeded(double v, const double *) { return (C)v; }
template <> __device__ inline Dual seeded<Dual>(double v, const double *t)
{
    Dual r(v);
    if (t) {
#pragma unroll
        for (int k = 0; k < kTangents; ++k) r.d[k] = t[k];
    }
    return r;
}

// periodic wrap of a coordinate (halos may span several periods of a tiny grid)
__device__ inline int wrap(int a, int n)
{
    a = a < 0 ? a + n : (a >= n ? a - n : a);
    if ((unsigned)a >= (unsigned)n) {
        while (a < 0) a += n;
        while (a >= n) a -= n;
    }
    return a;
}

__device__ inline bool solid_at(const RunDev &R, int x, int y)
{
    if (R.cyl_r <= 0) return false;
    const int dx = x - R.cyl_x, dy = y - R.cyl_y;
    return dx * dx + dy * dy <= R.cyl_r * R.cyl_r;
}

// A fluid node with a link into the cylinder lies within R + sqrt(2) of the centre; the test
// (R + 1)(R + 2) bounds that and keeps |x - x_c|, |y - y_c| <= R + 1 (the cut-link table's box).
__device__ inline bool near_cylinder(const RunDev &R, int x, int y)
{
    const int dx = x - R.cyl_x, dy = y - R.cyl_y;
    return R.cyl_r > 0 && dx * dx + dy * dy <= (R.cyl_r + 1) * (R.cyl_r + 2);
}

// Position kinds of the extended field: a node of the domain, an inlet ghost column (x < 0,
// rho/u of column 0, T = T_sat), a ghost behind the heated wall (x < 0 with the wall boundary:
// rho_w, u = 0, T_w, like a solid node) or an outlet ghost column (x >= nx, copy of column nx-1).
enum { NODE = 0, INLET_GHOST = 1, OUTLET_GHOST = 2, WALL_GHOST = 3 };

// (EXT: launches that carry the extended features, heated walls and phase-dependent properties;
// without it their code is absent)
template <bool EXT = true> __device__ inline int map_pos(const RunDev &R, int gx, int gy, int &rx, int &ry)
{
    ry = wrap(gy, R.ny);
    if (R.bc_x == 0) {
        rx = wrap(gx, R.nx);
        return NODE;
    }
    if (gx < 0) { rx = 0; return (EXT && R.bc_x == 2) ? WALL_GHOST : INLET_GHOST; }
    if (gx >= R.nx) { rx = R.nx - 1; return OUTLET_GHOST; }
    rx = gx;
    return NODE;
}

// ------------------------------------------------------------------------------------------
// Run constants in the compute type
// ------------------------------------------------------------------------------------------
template <typename C> struct Consts {
    C omega, sigma, gx, gy, rho_gref, rho_w, T_sat, T_w, a, b, Rg, u_in;
    C alpha, inv_cv, kappa, inv_sqrt_Tc, psi_scale, dphi_A, dphi_B;
    C alpha2w1, alpha2w2, alpha2w4, alpha2w5, alpha2w8;  // 2 alpha w_k of the Laplacian's weight classes
    C shiftw[9];
    // seed = false: tangent types take no parameter derivatives (plain constants)
    __device__ explicit Consts(const RunDev &R, bool seed = true)
    {
        omega = seeded<C>(R.omega, seed ? R.t_omega : nullptr); sigma = (C)R.sigma; gx = (C)R.gx; gy = (C)R.gy;
        rho_gref = (C)R.rho_gref; rho_w = (C)R.rho_w; T_sat = (C)R.T_sat;
        T_w = seeded<C>(R.T_w, seed ? R.t_T_w : nullptr);
        a = (C)R.eos_a; b = (C)R.eos_b; Rg = (C)R.eos_R; u_in = seeded<C>(R.u_in, seed ? R.t_u_in : nullptr);
        alpha = seeded<C>(R.alpha, seed ? R.t_alpha : nullptr); inv_cv = (C)R.inv_cv;
        kappa = seeded<C>(R.kappa, seed ? R.t_kappa : nullptr);
        inv_sqrt_Tc = (C)R.inv_sqrt_Tc;
        psi_scale = (C)R.psi_scale;
        // phi'(T) = dphi_A / sqrt(T) + dphi_B
        dphi_A = seeded<C>(R.dphi_A, seed ? R.t_dphi_A : nullptr);
        dphi_B = seeded<C>(R.dphi_B, seed ? R.t_dphi_B : nullptr);
        alpha2w1 = (C)(2.0 * W1) * alpha; alpha2w2 = (C)(2.0 * W2) * alpha; alpha2w4 = (C)(2.0 * W4) * alpha;
        alpha2w5 = (C)(2.0 * W5) * alpha; alpha2w8 = (C)(2.0 * W8) * alpha;
#pragma unroll
        for (int i = 0; i < 9; ++i) shiftw[i] = (C)(lat_w(i) * R.shift);
    }
};

// EOS-consistent pseudopotential (eq. potential) of the Peng-Robinson pressure (eq. eos)
template <typename C> __device__ inline C pseudopotential(const Consts<C> &K, C rho, C T)
{
    const C s = (C)1 + K.kappa * ((C)1 - Ar<C>::sqrt_(T) * K.inv_sqrt_Tc);
    const C phi = s * s;
    const C d1 = (C)1 - K.b * rho;
    const C d2 = (C)1 + (C)2 * K.b * rho - K.b * K.b * rho * rho;
    const C p = (rho * K.Rg * T * d2 - K.a * phi * rho * rho * d1) * Ar<C>::rcp(d1 * d2);
    return Ar<C>::sqrt_((p - rho * (C)(1.0 / 3.0)) * K.psi_scale);
}

// Phase-dependent transport (runs with phase_props): nu and alpha linear in density between the
// vapour and liquid coexistence densities, held constant outside that range.  PH: the launch
// carries the extended features (phase-dependent transport, heated walls); without it their code
// is compiled out.
template <typename C> __device__ inline C phase_frac(const RunDev &R, C rho, bool &inside)
{
    const C t = (rho - (C)R.rho_v) * (C)R.inv_drho;
    inside = t > (C)0 && t < (C)1;
    return t < (C)0 ? (C)0 : (t > (C)1 ? (C)1 : t);
}
// relaxation rate of the shear moments at density rho: 1 / (nu(rho) / cs^2 + 1/2)
template <bool PH, typename C> __device__ inline C omega_at(const RunDev &R, const Consts<C> &K, C rho)
{
    if constexpr (!PH) {
        return K.omega;
    } else {
        if (!R.phase_props) return K.omega;
        bool in;
        const C nu = (C)R.nu_v + phase_frac(R, rho, in) * (C)(R.nu_l - R.nu_v);
        return Ar<C>::rcp(nu * (C)3 + (C)0.5);
    }
}
// thermal diffusivity and its density derivative at density rho
template <bool PH, typename C> __device__ inline C alpha_at(const RunDev &R, const Consts<C> &K, C rho, C &dalpha)
{
    dalpha = (C)0;
    if (!PH || !R.phase_props) return K.alpha;
    bool in;
    const C t = phase_frac(R, rho, in);
    const C span = (C)(R.alpha - R.alpha_v);
    if (in) dalpha = span * (C)R.inv_drho;
    return (C)R.alpha_v + t * span;
}

// ------------------------------------------------------------------------------------------
// Central-moment collision of one node (eq. posColl0 with the corrected moments of eq. postColl2,
// reconstructed as f* = M^-1 N(-u) k*, Appendix A) from its density rho, momentum (jx, jy), raw
// second moments m4 = sum f (cx^2 - cy^2), m5 = sum f cx cy, total force (Fx, Fy), the consistency
// term A = 2 sigma |F_m|^2 / psi^2 and the shear relaxation rate om.  Returns the velocity
// u = (j + F/2) / rho in (U, V); fs receives f*_1..8, and f*_0 closes the mass balance.
// ------------------------------------------------------------------------------------------
template <typename C>
__device__ __forceinline__ void collide_node(C rho, C jx, C jy, C m4, C m5, C Fx, C Fy, C A, C om, C &U, C &V,
                                             C fs[9])
{
    const C ir = Ar<C>::rcp(rho);
    U = (jx + (C)0.5 * Fx) * ir;
    V = (jy + (C)0.5 * Fy) * ir;
    // pre-collision central moments k4, k5 from raw moments (rows 4, 5 of N(u))
    const C k4 = (U * U - V * V) * rho - (C)2 * U * jx + (C)2 * V * jy + m4;
    const C k5 = U * V * rho - V * jx - U * jy + m5;
    // post-collision central moments (eq. postColl2)
    const C k0 = rho, k1 = (C)0.5 * Fx, k2 = (C)0.5 * Fy;
    const C k3 = (C)(2.0 / 3.0) * rho + A;
    const C k4s = ((C)1 - om) * k4, k5s = ((C)1 - om) * k5;
    const C k6 = Fy * (C)(1.0 / 6.0), k7 = Fx * (C)(1.0 / 6.0);
    const C k8 = rho * (C)(1.0 / 9.0) + A * (C)(1.0 / 3.0);
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
    // populations f* = M^-1 m*; f*_0 closes the mass balance sum_i f*_i = k*_0 = rho exactly
    fs[1] = (C)0.5 * (r1 - r7 - r8) + (C)0.25 * (r3 + r4);
    fs[2] = (C)0.5 * (-r1 + r7 - r8) + (C)0.25 * (r3 + r4);
    fs[3] = (C)0.5 * (r2 - r6 - r8) + (C)0.25 * (r3 - r4);
    fs[4] = (C)0.5 * (-r2 + r6 - r8) + (C)0.25 * (r3 - r4);
    fs[5] = (C)0.25 * (r5 + r6 + r7 + r8);
    fs[6] = (C)0.25 * (r5 - r6 - r7 + r8);
    fs[7] = (C)0.25 * (-r5 - r6 + r7 + r8);
    fs[8] = (C)0.25 * (-r5 + r6 - r7 + r8);
    fs[0] = r0 - (((fs[1] + fs[2]) + (fs[3] + fs[4])) + ((fs[5] + fs[6]) + (fs[7] + fs[8])));
}

}  // namespace
}  // namespace lbm
