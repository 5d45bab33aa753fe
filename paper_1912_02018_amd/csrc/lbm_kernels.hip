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
//              carrying a halo of 2 nodes per stage so the stages never leave the CU; positions
//              are updated in vertically adjacent pairs that share their stencil rows
//              (k_thermal_tan: the same step for the tangent precision, one position at a time).
//   k_diag_*   FP64 mass and wall heat-flux reductions in a fixed order (bitwise reproducible).
//   k_init     f* := f^eq(rho, u), outlet history, temperature from host-provided fields.
// No MFMA: every kernel is a stencil or an elementwise map.  The 24-neighbour stencils are
// evaluated on sums and differences of opposite neighbours, grouped by weight class.

#include "lbm_device.h"

#include <hip/hip_ext.h>

#include <map>
#include <mutex>

namespace lbm {
namespace {

// ------------------------------------------------------------------------------------------
// Streaming of one fluid node: f_i(x) = f*_i(x - c_i) with the boundary conditions
// ------------------------------------------------------------------------------------------
// Load population i at element offset (i * plane + y * pitch + x) of a population buffer.  The
// byte offset is formed in 32 bits (9 planes stay below 4 GiB) so that the load takes the
// scalar-base + 32-bit vector-offset form.
template <typename S, typename C>
__device__ inline C ldf(const char *base, unsigned plane, unsigned pitch, int i, int x, int y, const Consts<C> &K)
{
    const unsigned off = ((unsigned)i * plane + (unsigned)y * pitch + (unsigned)x) * (unsigned)sizeof(RawT<S>);
    return Conv<S>::ld(*(gp<const RawT<S>>)(base + off), K.shiftw[i]);
}

// Plain pulls of a node away from the cylinder; at the inlet / outlet columns the sources outside
// the domain are clamped in (apply_x_bc then replaces the inlet's unknowns; at the outlet the clamped
// values are the ones the convective condition needs).  Offsets are formed once per node: one row
// product, neighbouring rows and columns by adds and selects.
template <typename S, typename C, bool EXT = true>
__device__ inline void pull_bulk(const RunDev &R, const Consts<C> &K, const char *fin, int x, int y, C f[9])
{
    constexpr unsigned es = (unsigned)sizeof(RawT<S>);
    const int nx = R.nx, ny = R.ny, P = R.pitch;
    const unsigned rowB = (unsigned)P * es, planeB = (unsigned)ny * rowB;
    const bool periodic = R.bc_x == 0;
    const unsigned r0 = (unsigned)y * rowB;
    const unsigned rm = y == 0 ? r0 + planeB - rowB : r0 - rowB;
    const unsigned rp = y == ny - 1 ? r0 + rowB - planeB : r0 + rowB;
    const unsigned c0 = (unsigned)x * es;
    const unsigned cm = x == 0 ? (periodic ? (unsigned)(nx - 1) * es : 0u) : c0 - es;
    const unsigned cp = x == nx - 1 ? (periodic ? 0u : c0) : c0 + es;
    // next to the heated wall at x = -1/2 (halfway bounce-back) the populations entering along
    // +x are the node's own outgoing ones reversed: f_i(0, y) = f*_opp(i)(0, y)
    const bool wall = EXT && R.bc_x == 2 && x == 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        unsigned row = cy_of(i) > 0 ? rm : (cy_of(i) < 0 ? rp : r0);
        const unsigned col = cx_of(i) > 0 ? cm : (cx_of(i) < 0 ? cp : c0);
        unsigned plane = (unsigned)i * planeB;
        if (cx_of(i) > 0) {
            row = wall ? r0 : row;
            plane = wall ? (unsigned)opp_of(i) * planeB : plane;
        }
        // (opposite directions share the lattice weight, so the storage shift of i applies)
        f[i] = Conv<S>::ld(*(gp<const RawT<S>>)(fin + (plane + row + col)), K.shiftw[i]);
    }
}

// Links of a node next to the cylinder whose source is solid: linear interpolated bounce-back on
// the curved wall.  The wall fraction of every cut link is tabulated on the host over the box
// |x - x_c|, |y - y_c| <= R + 1 (8 entries per node, directions 1..8):
//   0          the source is fluid: the plain pull stands
//   v in (0,1) q < 1/2 with a fluid node at x + c_i:  f_i = v f*_o(x) + (1 - v) f*_o(x + c_i), v = 2q
//   v > 2      q < 1/2 without one:                    f_i = f*_o(x)
//   v <= -1    q >= 1/2:                              f_i = f*_o(x)/(2q) + (2q - 1)/(2q) f*_i(x), v = -2q
// f*_o(x + c_i) is the plain pull of direction o = opp(i): the box keeps one node clear of every
// domain edge, so that pull is neither wrapped nor clamped, and only the wall fractions and the
// node's own populations are loaded.
template <typename S, typename C>
__device__ inline void fix_near(const RunDev &R, const Consts<C> &K, const char *fin, int x, int y, C f[9])
{
    const unsigned P = R.pitch, plane = (unsigned)R.ny * P;
    const int bw = 2 * R.cyl_r + 3;
    const C *qt = (const C *)R.qtab + ((y - (R.cyl_y - R.cyl_r - 1)) * bw + (x - (R.cyl_x - R.cyl_r - 1))) * 8;
    // every operand is loaded up front (one round trip), then each link selects its rule
    C v[9], own[9], nb[9];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        v[i] = qt[i - 1];
        own[i] = ldf<S, C>(fin, plane, P, i, x, y, K);
        nb[i] = f[opp_of(i)];
    }
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const C fo = own[opp_of(i)];
        const C q2 = -v[i];
        const C lt = v[i] * fo + ((C)1 - v[i]) * nb[i];
        const C ge = fo / q2 + (q2 - (C)1) / q2 * own[i];
        f[i] = v[i] == (C)0 ? f[i] : (v[i] > (C)2 ? fo : (v[i] > (C)0 ? lt : ge));
    }
}

// Velocity inlet at x = 0 and convective outlet at x = nx - 1 (the heated wall's bounce-back is
// part of the plain pulls).  EXT: the launch carries the extended features, among them the outlet
// speed taken from the local outflow.
template <typename S, typename C, bool EXT = true>
__device__ inline void apply_x_bc(const RunDev &R, const Consts<C> &K, const char *fin, gp<const C> hin, int x, int y,
                                  C f[9])
{
    const int nx = R.nx, ny = R.ny;
    if (x == nx - 1) {
        // convective outflow: f^{n+1}(N) = (f^n(N) + U f^{n+1}(N-1)) / (1 + U), i in {2,6,8}.  The
        // plain pulls of column N clamp their x source to N, so f[2], f[6], f[8] already hold
        // f*_2(N, y), f*_6(N, y + 1), f*_8(N, y - 1): the populations that stream into N - 1.
        C U = K.u_in;
        if (EXT && R.outlet_kind == 1) {
            // local outflow speed: x velocity of the node's own post-collision populations (the
            // previous time level), none where the flow turns back in
            const unsigned P = R.pitch, plane = (unsigned)R.ny * P;
            C m = 0, jx = 0;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const C fi = ldf<S, C>(fin, plane, P, i, x, y, K);
                m = m + fi;
                jx = jx + (C)cx_of(i) * fi;
            }
            U = jx / m;
            U = U > (C)0 ? U : (C)0;
        }
        const C inv = Ar<C>::rcp((C)1 + U);
        const C p2 = f[2], p6 = f[6], p8 = f[8];
        f[2] = (hin[0 * ny + y] + U * p2) * inv;
        f[6] = (hin[1 * ny + y] + U * p6) * inv;
        f[8] = (hin[2 * ny + y] + U * p8) * inv;
    }
    if (x == 0 && R.bc_x != 2) {
        // velocity inlet (u_in, 0): unknowns 1, 5, 7
        const C u = K.u_in;
        const C rin = (f[0] + f[3] + f[4] + (C)2 * (f[2] + f[6] + f[8])) * Ar<C>::rcp((C)1 - u);
        f[1] = f[2] + (C)(2.0 / 3.0) * rin * u;
        f[5] = f[6] - (C)0.5 * (f[3] - f[4]) + rin * u * (C)(1.0 / 6.0);
        f[7] = f[8] + (C)0.5 * (f[3] - f[4]) + rin * u * (C)(1.0 / 6.0);
    }
}

// Corrections of the plain pulls f of a node next to the cylinder or on an inlet / outlet column.
template <typename S, typename C, bool EXT = true>
__device__ inline void fix_special(const RunDev &R, const Consts<C> &K, const char *fin, const void *hin, int x, int y,
                                   C f[9])
{
    if (near_cylinder(R, x, y)) fix_near<S, C>(R, K, fin, x, y, f);
    if (R.bc_x != 0 && (x == 0 || x == R.nx - 1)) apply_x_bc<S, C, EXT>(R, K, fin, gin<C>(hin), x, y, f);
}

// An index the optimiser cannot re-associate with the constant offsets added to it afterwards,
// so that a 5x5 LDS window is read with one base register and immediate offsets.
__device__ inline int opaque_index(int i)
{
    asm volatile("" : "+v"(i));
    return i;
}

// x and y components of sum_k w_k a(x + e_k) e_k from the differences of opposite neighbours
template <typename C> struct PairD {
    C d10, d01, d11, d1m, d20, d02, d21, d2m, d12, d1m2, d22, d2m2;
    __device__ C gx() const
    {
        return (C)W1 * d10 + (C)W2 * (d11 + d1m) + (C)(2 * W4) * d20 + (C)W5 * ((C)2 * (d21 + d2m) + d12 + d1m2) +
               (C)(2 * W8) * (d22 + d2m2);
    }
    __device__ C gy() const
    {
        return (C)W1 * d01 + (C)W2 * (d11 - d1m) + (C)(2 * W4) * d02 + (C)W5 * (d21 - d2m + (C)2 * (d12 - d1m2)) +
               (C)(2 * W8) * (d22 - d2m2);
    }
};

// differences of opposite neighbours of LDS position c in a row-major array of row stride RW
// (addressed from the lowest corner of the 5x5 window so that every read is a positive offset
// from one base address)
template <int RW, typename C> __device__ inline PairD<C> pair_diffs(const C *s, int c)
{
    const C *b = s + opaque_index(c - 2 * RW - 2);
#define W_(dx, dy) b[(2 + (dy)) * RW + 2 + (dx)]
    PairD<C> d;
    d.d10 = W_(1, 0) - W_(-1, 0);
    d.d01 = W_(0, 1) - W_(0, -1);
    d.d11 = W_(1, 1) - W_(-1, -1);
    d.d1m = W_(1, -1) - W_(-1, 1);
    d.d20 = W_(2, 0) - W_(-2, 0);
    d.d02 = W_(0, 2) - W_(0, -2);
    d.d21 = W_(2, 1) - W_(-2, -1);
    d.d2m = W_(2, -1) - W_(-2, 1);
    d.d12 = W_(1, 2) - W_(-1, -2);
    d.d1m2 = W_(1, -2) - W_(-1, 2);
    d.d22 = W_(2, 2) - W_(-2, -2);
    d.d2m2 = W_(2, -2) - W_(-2, 2);
#undef W_
    return d;
}

// ------------------------------------------------------------------------------------------
// k_lbm: streaming + moments + psi + force + central-moment collision
// ------------------------------------------------------------------------------------------
// OCC > 0: ask the compiler for at least OCC waves per SIMD (a register budget)
template <typename S, int TX, int TY, int NT, bool WRITE_F, bool PH, int OCC = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1))) void k_lbm(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles, int pf,
                                            int pt, int ph, long long step)
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
    const char *fin = (const char *)R.f[pf];
    char *fout = (char *)R.f[pf ^ 1];
    const gp<C> hout = gout<C>(R.hist[ph ^ 1]);

    // phase 1: density (and psi) on the tile plus halo, raw moments on the tile.  Each thread
    // first issues the pull loads of all its positions so that they are in flight together, then
    // corrects the positions next to the cylinder or on the inlet / outlet columns.
    constexpr int IT1 = (RN + NT - 1) / NT;
    C fv[IT1][9];
    C Tv[IT1];
    int rxv[IT1], ryv[IT1];
    unsigned need = 0, solid = 0, inlet = 0;
#pragma unroll
    for (int j = 0; j < IT1; ++j) {
        const int p = threadIdx.x + NT * j;
        if (p >= RN) continue;
        const int lx = p % RW, ly = p / RW;
        const int gx = x0 - H + lx, gy = y0 - H + ly;
        const bool own = lx >= H && lx < H + TX && ly >= H && ly < H + TY && gx < nx && gy < ny;
        if (!fon && !own) continue;
        int rx, ry;
        const int kind = map_pos<PH>(R, gx, gy, rx, ry);
        rxv[j] = rx;
        ryv[j] = ry;
        need |= 1u << j;
        if (kind == INLET_GHOST) inlet |= 1u << j;
        if (kind == WALL_GHOST || solid_at(R, rx, ry)) {
            solid |= 1u << j;
            continue;
        }
        pull_bulk<S, C, PH>(R, K, fin, rx, ry, fv[j]);
        Tv[j] = ld_at<C>(R.T[pt], (unsigned)(ry * P + rx));
    }
#pragma unroll
    for (int j = 0; j < IT1; ++j) {
        if (!((need >> j) & 1u)) continue;
        const int p = threadIdx.x + NT * j;
        const int lx = p % RW, ly = p / RW;
        const int gx = x0 - H + lx, gy = y0 - H + ly;
        const bool own = lx >= H && lx < H + TX && ly >= H && ly < H + TY && gx < nx && gy < ny;
        const int rx = rxv[j], ry = ryv[j];
        const int q = (ly - H) * TX + (lx - H);
        C rho, T;
        if ((solid >> j) & 1u) {
            rho = K.rho_w;
            T = K.T_w;
            if (own) { s_m[0][q] = rho; s_m[1][q] = 0; s_m[2][q] = 0; s_m[3][q] = 0; s_m[4][q] = 0; }
        } else {
            C *f = fv[j];
            if (near_cylinder(R, rx, ry) || (R.bc_x != 0 && (rx == 0 || rx == nx - 1)))
                fix_special<S, C, PH>(R, K, fin, R.hist[ph], rx, ry, f);
            rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
            T = ((inlet >> j) & 1u) ? K.T_sat : Tv[j];
            if (own) {
                s_m[0][q] = rho;
                s_m[1][q] = (f[1] - f[2]) + (f[5] - f[6]) + (f[7] - f[8]);
                s_m[2][q] = (f[3] - f[4]) + (f[5] - f[6]) + (f[8] - f[7]);
                s_m[3][q] = (f[1] + f[2]) - (f[3] + f[4]);
                s_m[4][q] = (f[5] + f[6]) - (f[7] + f[8]);
                if (WRITE_F && R.bc_x != 0 && gx == nx - 1) {
                    hout[0 * ny + gy] = f[2];
                    hout[1 * ny + gy] = f[6];
                    hout[2 * ny + gy] = f[8];
                }
            }
        }
        if (fon) s_psi[p] = pseudopotential(K, rho, T);
    }
    __syncthreads();

    const unsigned plane = (unsigned)ny * P;

    // phase 2: force, velocity, collision of the tile nodes
    for (int q = threadIdx.x; q < TN; q += NT) {
        const int lx = q % TX, ly = q / TX;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= nx || gy >= ny) continue;
        const unsigned idx = (unsigned)(gy * P + gx);
        if (solid_at(R, gx, gy)) {
            *at<C>(R.rho, idx) = K.rho_w;
            *at<C>(R.ux, idx) = 0;
            *at<C>(R.uy, idx) = 0;
            // never streamed from, but kept deterministic: the rest state of the wall density
            if (WRITE_F) {
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    *(gp<RawT<S>>)(fout + ((unsigned)i * (unsigned)plane + (unsigned)idx) * (unsigned)sizeof(RawT<S>)) =
                        Conv<S>::st((C)lat_w(i) * K.rho_w, K.shiftw[i]);
            }
            continue;
        }
        const C rho = s_m[0][q], jx = s_m[1][q], jy = s_m[2][q], m4 = s_m[3][q], m5 = s_m[4][q];
        C Fx = 0, Fy = 0, A = 0;
        if (fon) {
            const int c = (ly + H) * RW + (lx + H);
            const PairD<C> d = pair_diffs<RW>(s_psi, c);
            const C psi0 = s_psi[c];
            // F_m = -G cs^2 psi sum_k w_k psi(x + e_k) e_k (eq. interForce); G cs^2 = 2/psi_scale
            const C pre = -(C)2 * Ar<C>::rcp(K.psi_scale) * psi0;
            const C Fmx = pre * d.gx();
            const C Fmy = pre * d.gy();
            A = (C)2 * K.sigma * (Fmx * Fmx + Fmy * Fmy) * Ar<C>::rcp(psi0 * psi0);
            Fx = Fmx + (rho - K.rho_gref) * K.gx;
            Fy = Fmy + (rho - K.rho_gref) * K.gy;
        }
        C U, V, fs[9];
        collide_node<C>(rho, jx, jy, m4, m5, Fx, Fy, A, omega_at<PH>(R, K, rho), U, V, fs);
        *at<C>(R.rho, idx) = rho;
        *at<C>(R.ux, idx) = U;
        *at<C>(R.uy, idx) = V;
        if (!WRITE_F) continue;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            *(gp<RawT<S>>)(fout + ((unsigned)i * (unsigned)plane + (unsigned)idx) * (unsigned)sizeof(RawT<S>)) =
                Conv<S>::st(fs[i], K.shiftw[i]);
    }
}

// ------------------------------------------------------------------------------------------
// k_lbm_strip: the same step for a strip of NT - 4 columns marching down a chunk of CH rows
// ------------------------------------------------------------------------------------------
// Lane l owns column x0 - 2 + l.  An iteration forms the pulls, moments and psi of 4 rows q .. q + 3
// (all lanes: the strip and 2 halo columns on each side; every pull of the 4 rows is issued before
// the first is used) and collides rows q - 2 .. q + 1 (the strip's columns) with the psi of rows
// q - 4 .. q + 3 from a ring of 12 LDS rows, so that every position's pulls and psi are formed once
// per chunk instead of once per tile that reaches it (a 64 x 8 tile forms psi on 68 x 12 positions).
// One barrier per iteration: the ring holds the rows the collision reads plus the 4 written next.
// The per-node arithmetic is that of k_lbm, so both give the same bits.
template <typename C> __device__ inline PairD<C> pair_diffs_rows(const C *const rows[5], int c)
{
#define W_(dx, dy) rows[2 + (dy)][c + (dx)]
    PairD<C> d;
    d.d10 = W_(1, 0) - W_(-1, 0);
    d.d01 = W_(0, 1) - W_(0, -1);
    d.d11 = W_(1, 1) - W_(-1, -1);
    d.d1m = W_(1, -1) - W_(-1, 1);
    d.d20 = W_(2, 0) - W_(-2, 0);
    d.d02 = W_(0, 2) - W_(0, -2);
    d.d21 = W_(2, 1) - W_(-2, -1);
    d.d2m = W_(2, -1) - W_(-2, 1);
    d.d12 = W_(1, 2) - W_(-1, -2);
    d.d1m2 = W_(1, -2) - W_(-1, 2);
    d.d22 = W_(2, 2) - W_(-2, -2);
    d.d2m2 = W_(2, -2) - W_(-2, 2);
#undef W_
    return d;
}

template <typename S, int NT, int CH, bool WRITE_F, bool PH, int OCC = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1))) void k_lbm_strip(
    const RunDev *__restrict__ runs, const Tile *__restrict__ tiles, int pf, int pt, int ph, long long step)
{
    using C = CT<S>;
    constexpr int W = NT - 4, RB = 4, RING = 3 * RB;
    static_assert(CH % RB == 0, "chunks are whole groups of rows");
    __shared__ C s_psi[RING][NT];

    const Tile t = tiles[blockIdx.x];
    const RunDev &R = runs[t.run];
    const Consts<C> K(R);
    const int nx = R.nx, ny = R.ny, P = R.pitch;
    const bool fon = step >= R.warmup;
    const char *fin = (const char *)R.f[pf];
    char *fout = (char *)R.f[pf ^ 1];
    const gp<C> hout = gout<C>(R.hist[ph ^ 1]);
    const int lane = threadIdx.x;
    const int gx = t.tx * W - 2 + lane;
    const bool own_col = lane >= 2 && lane < NT - 2 && gx < nx;
    const int y0 = t.ty * CH, y1 = min(ny, y0 + CH);
    const unsigned plane = (unsigned)ny * P;
    // the kind of a position and its mapped column depend on the column only
    int rx, ry_;
    const int kind = map_pos<PH>(R, gx, 0, rx, ry_);

    // iteration: rows q .. q + RB - 1 (pulls, moments, psi; all lanes), then rows q - 2 .. q + RB - 3
    // (force and collision; the strip's columns) with the psi of rows q - 4 .. q + RB - 1.  The raw
    // moments (rho, jx, jy, sum f (cx^2 - cy^2), sum f cx cy) stay with the lane that formed them: rows
    // q, q + 1 are collided in the same iteration, rows q + 2, q + 3 in the next (mprev).
    C mprev[2][5] = {};
    for (int q = y0 - 2, it = 0; q - 2 < y1; q += RB, ++it) {
        C mcur[RB][5] = {};
        C f[RB][9], Tv[RB];
        unsigned skip = 0;   // bit j: row q + j forms nothing (outside the chunk's reach, or solid)
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const int y = q + j;
            const bool own_row = y >= y0 && y < y1;
            const int ry = wrap(y, ny);
            if (y >= y1 + 2 || !(fon || (own_col && own_row)) || kind == WALL_GHOST || solid_at(R, rx, ry)) {
                skip |= 1u << j;
                continue;
            }
            pull_bulk<S, C, PH>(R, K, fin, rx, ry, f[j]);
            Tv[j] = ld_at<C>(R.T[pt], (unsigned)(ry * P + rx));
        }
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const int y = q + j;
            const bool own_row = y >= y0 && y < y1;
            if (y >= y1 + 2 || !(fon || (own_col && own_row))) continue;
            const int ry = wrap(y, ny);
            C rho, T, m[5];
            if ((skip >> j) & 1u) {
                rho = K.rho_w;
                T = K.T_w;
                m[0] = rho; m[1] = 0; m[2] = 0; m[3] = 0; m[4] = 0;
            } else {
                C *fj = f[j];
                if (near_cylinder(R, rx, ry) || (R.bc_x != 0 && (rx == 0 || rx == nx - 1)))
                    fix_special<S, C, PH>(R, K, fin, R.hist[ph], rx, ry, fj);
                rho = ((fj[0] + fj[1]) + (fj[2] + fj[3])) + ((fj[4] + fj[5]) + (fj[6] + fj[7])) + fj[8];
                T = kind == INLET_GHOST ? K.T_sat : Tv[j];
                m[0] = rho;
                m[1] = (fj[1] - fj[2]) + (fj[5] - fj[6]) + (fj[7] - fj[8]);
                m[2] = (fj[3] - fj[4]) + (fj[5] - fj[6]) + (fj[8] - fj[7]);
                m[3] = (fj[1] + fj[2]) - (fj[3] + fj[4]);
                m[4] = (fj[5] + fj[6]) - (fj[7] + fj[8]);
                if (WRITE_F && own_col && own_row && R.bc_x != 0 && gx == nx - 1) {
                    hout[0 * ny + y] = fj[2];
                    hout[1 * ny + y] = fj[6];
                    hout[2 * ny + y] = fj[8];
                }
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) mcur[j][k] = m[k];
            if (fon) s_psi[(it % 3) * RB + j][lane] = pseudopotential(K, rho, T);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const int r = q - 2 + j;
            if (r < y0 || r >= y1 || !own_col) continue;
            const unsigned idx = (unsigned)(r * P + gx);
            if (solid_at(R, gx, r)) {
                *at<C>(R.rho, idx) = K.rho_w;
                *at<C>(R.ux, idx) = 0;
                *at<C>(R.uy, idx) = 0;
                if (WRITE_F) {
#pragma unroll
                    for (int i = 0; i < 9; ++i)
                        *(gp<RawT<S>>)(fout + ((unsigned)i * plane + idx) * (unsigned)sizeof(RawT<S>)) =
                            Conv<S>::st((C)lat_w(i) * K.rho_w, K.shiftw[i]);
                }
                continue;
            }
            // row r was formed in this iteration (j >= 2) or in the previous one (j < 2)
            const C *mr = j >= 2 ? mcur[j - 2] : mprev[j];
            const C rho = mr[0], jx = mr[1], jy = mr[2], m4 = mr[3], m5 = mr[4];
            C Fx = 0, Fy = 0, A = 0;
            if (fon) {
                // psi of rows r - 2 .. r + 2: the ring slot of row q + i is ((it + (i < 0 ? -1 : 0)) mod 3) RB + i mod RB
                const C *rows[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    const int i = j - 4 + k;   // row r - 2 + k = q + i, i in -4 .. RB - 1
                    const int itr = i < 0 ? it - 1 : it;
                    rows[k] = s_psi[(itr % 3) * RB + (i < 0 ? i + RB : i)];
                }
                const PairD<C> d = pair_diffs_rows(rows, lane);
                const C psi0 = rows[2][lane];
                // F_m = -G cs^2 psi sum_k w_k psi(x + e_k) e_k (eq. interForce); G cs^2 = 2/psi_scale
                const C pre = -(C)2 * Ar<C>::rcp(K.psi_scale) * psi0;
                const C Fmx = pre * d.gx();
                const C Fmy = pre * d.gy();
                A = (C)2 * K.sigma * (Fmx * Fmx + Fmy * Fmy) * Ar<C>::rcp(psi0 * psi0);
                Fx = Fmx + (rho - K.rho_gref) * K.gx;
                Fy = Fmy + (rho - K.rho_gref) * K.gy;
            }
            C U, V, fs[9];
            collide_node<C>(rho, jx, jy, m4, m5, Fx, Fy, A, omega_at<PH>(R, K, rho), U, V, fs);
            *at<C>(R.rho, idx) = rho;
            *at<C>(R.ux, idx) = U;
            *at<C>(R.uy, idx) = V;
            if (!WRITE_F) continue;
#pragma unroll
            for (int i = 0; i < 9; ++i)
                *(gp<RawT<S>>)(fout + ((unsigned)i * plane + idx) * (unsigned)sizeof(RawT<S>)) =
                    Conv<S>::st(fs[i], K.shiftw[i]);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            mprev[0][k] = mcur[2][k];
            mprev[1][k] = mcur[3][k];
        }
    }
}

// ------------------------------------------------------------------------------------------
// k_thermal: Runge-Kutta update of the temperature equation (eq. energy) for one tile
// ------------------------------------------------------------------------------------------
// The temperature kernels (to the tangent kernel below) let the compiler fuse a multiply with a
// later add across statements, as the rest of the library does only within one expression: their
// tile and strip variants are pinned to the same bits by the variant tests (their inputs are FP32
// or FP64 in every storage format), and the fusions take 4 % off the strip's time on large grids.
#pragma clang fp contract(fast)
// The frozen fields rho, u and T^n are loaded with a halo of 2 nodes per stage, so the stages
// never leave the CU: stage s updates the tile grown by 2 (NS - s) nodes.  Each thread owns a
// fixed set of slots for the whole kernel, a slot being two vertically adjacent positions, and
// keeps their stage-invariant coefficients in registers (T^n and the Runge-Kutta accumulator too,
// unless the thread has many slots); LDS holds the stage inputs and rho, u for the invariants.
// A slot reads the 6 x 5 window of its two positions once and forms the row sums and differences
// that both positions' stencils are built from.  Slots are numbered ring by ring outwards from the tile (the halo of a
// stage is 2 nodes, so every ring is made of whole pairs), so the slots of a later, smaller stage
// are a prefix of the numbering and whole wavefronts drop out as the stages shrink.
template <int TX, int TY, int NS> struct ThGeom {
    static_assert(TY % 2 == 0, "slots pair the rows of the tile");
    static constexpr int H = 2 * NS;
    // region of RX x RH positions stored with an odd row stride RW (the ring slots of a wavefront
    // are short row pieces a stride apart, which an even stride would put on few LDS banks)
    static constexpr int RX = TX + 2 * H, RW = RX + 1, RH = TY + 2 * H, RN = RW * RH, TN = TX * TY;
    // slots updated by stage s
    static constexpr int count(int s) { return (TX + 4 * (NS - s)) * (TY + 4 * (NS - s)) / 2; }
    static constexpr int NSLOT = count(1), TSLOT = TN / 2;
};

template <int TX, int TY, int NS> struct SlotTable {
    unsigned short pos[ThGeom<TX, TY, NS>::NSLOT];  // LDS position of the slot's upper node
};

template <int TX, int TY, int NS> constexpr SlotTable<TX, TY, NS> make_slots()
{
    using G = ThGeom<TX, TY, NS>;
    SlotTable<TX, TY, NS> t{};
    int r = 0;
    for (int yp = 0; yp < TY / 2; ++yp)
        for (int x = 0; x < TX; ++x) t.pos[r++] = (unsigned short)((G::H + 2 * yp) * G::RW + G::H + x);
    // ring k: the tile grown by 2k nodes minus the tile grown by 2(k - 1); its top and bottom
    // bands are one row of pairs each, its sides columns of pairs
    for (int k = 1; k < NS; ++k) {
        const int o = G::H - 2 * k, A = TX + 4 * (k - 1), B = TY + 4 * (k - 1);
        for (int xx = 0; xx < A + 4; ++xx) t.pos[r++] = (unsigned short)(o * G::RW + o + xx);
        for (int xx = 0; xx < A + 4; ++xx) t.pos[r++] = (unsigned short)((o + B + 2) * G::RW + o + xx);
        for (int yp = 0; yp < B / 2; ++yp)
            for (int q = 0; q < 4; ++q) t.pos[r++] = (unsigned short)((o + 2 + 2 * yp) * G::RW + o + (q < 2 ? q : A + q));
    }
    return t;
}

template <int TX, int TY, int NS> __constant__ const SlotTable<TX, TY, NS> kSlots = make_slots<TX, TY, NS>();

// Sums and differences of opposite neighbours along one row of a 5-wide window (r: its column -2):
// h0 = a(0), s1 = a(1) + a(-1), s2 = a(2) + a(-2), d1 = a(1) - a(-1), d2 = a(2) - a(-2)
template <typename C> struct RowQ {
    C h0, s1, s2, d1, d2;
};
template <typename C> __device__ inline RowQ<C> row_q(const C *r)
{
    return RowQ<C>{r[2], r[3] + r[1], r[4] + r[0], r[3] - r[1], r[4] - r[0]};
}

// x and y components of sum_k w_k a(x + e_k) e_k at the node of row q[2] (q: rows -2 .. 2), the
// opposite-neighbour pairs of each weight class grouped by rows
template <typename C> __device__ inline C grad_x(const RowQ<C> *q)
{
    return (C)W1 * q[2].d1 + (C)(2 * W4) * q[2].d2 + (C)W2 * (q[3].d1 + q[1].d1) + (C)(2 * W5) * (q[3].d2 + q[1].d2) +
           (C)W5 * (q[4].d1 + q[0].d1) + (C)(2 * W8) * (q[4].d2 + q[0].d2);
}
template <typename C> __device__ inline C grad_y(const RowQ<C> *q)
{
    return (C)W1 * (q[3].h0 - q[1].h0) + (C)(2 * W4) * (q[4].h0 - q[0].h0) + (C)W2 * (q[3].s1 - q[1].s1) +
           (C)W5 * (q[3].s2 - q[1].s2) + (C)(2 * W5) * (q[4].s1 - q[0].s1) + (C)(2 * W8) * (q[4].s2 - q[0].s2);
}

// Coefficients of L(Y) at the two nodes of a slot ([n]: upper / lower; 8 per node): u/12, v/12
// and |u| c_d, |v| c_d of the upwind convection, the density-gradient coefficients gx, gy, the
// centre coefficient c0 (the Laplacian's and the convection's centre weights and the linear part c1
// of the source) and c2 of sqrt(Y)
template <typename C, bool PH> struct ThCoef {
    C u12[2], v12[2], au[2], av[2], gx[2], gy[2], c0[2], c2[2];
    C al[PH ? 2 : 1];  // alpha at the node (phase-dependent properties)
};

// Stage-invariant coefficients of both nodes of a slot from the 6 x 5 windows of rho, u_x and u_y
// (rr[k], ru[k], rv[k]: column -2 of window row k, rows -2 .. 3 of the upper node).  Bit n of hj
// marks a solid node, whose coefficients are left as they are.  The windows are read one field at a
// time (its window, then the stencils it feeds), which bounds the registers they hold.
//   gx, gy = alpha grad(rho)/rho;  source(T) = c1 T + c2 sqrt(T) with
//   D = div(u)/(rho cv), c1 = -D R rho/(1 - b rho) + B D a rho^2/(1 + 2 b rho - b^2 rho^2),
//   c2 = A D a rho^2/(1 + 2 b rho - b^2 rho^2), phi'(T) = A/sqrt(T) + B
template <typename C, bool PH>
__device__ __forceinline__ void thermal_coef(const RunDev &R, const Consts<C> &K, const C *const rr[6],
                                             const C *const ru[6], const C *const rv[6], unsigned hj, C cd,
                                             ThCoef<C, PH> &f)
{
    C rho[2], gxr[2], gyr[2], u[2], v[2], div[2];
    {
        RowQ<C> q[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) q[k] = row_q(rr[k]);
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            rho[n] = q[n + 2].h0;
            gxr[n] = grad_x(q + n);
            gyr[n] = grad_y(q + n);
        }
    }
    {
        RowQ<C> q[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) q[k] = row_q(ru[k]);
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            u[n] = q[n + 2].h0;
            div[n] = grad_x(q + n);
        }
    }
    {
        RowQ<C> q[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) q[k] = row_q(rv[k]);
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            v[n] = q[n + 2].h0;
            div[n] = div[n] + grad_y(q + n);
        }
    }
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        if ((hj >> n) & 1u) continue;
        const C ir = Ar<C>::rcp(rho[n]);
        // (1/(rho cv)) div(lambda grad T) with lambda = rho cv alpha(rho):
        //   alpha (lap T + grad rho . grad T / rho) + alpha'(rho) grad rho . grad T
        C dal;
        const C al = alpha_at<PH>(R, K, rho[n], dal);
        const C gcoef = al * ir + dal;
        const C gx = gcoef * gxr[n];
        const C gy = gcoef * gyr[n];
        const C D = div[n] * ir * K.inv_cv;
        const C d1 = (C)1 - K.b * rho[n];
        const C d2 = (C)1 + (C)2 * K.b * rho[n] - K.b * K.b * rho[n] * rho[n];
        const C A2 = D * K.a * rho[n] * rho[n] * Ar<C>::rcp(d2);
        const C c1 = -D * rho[n] * K.Rg * Ar<C>::rcp(d1) + K.dphi_B * A2;
        f.c2[n] = K.dphi_A * A2;
        // third-order upwind-biased convection per axis:
        //   u (8 d1 - d2) / 12 + |u| c_d (S2 - 4 S1 + 6 Y)   (d, S: differences / sums of the pair)
        const C au = absval(u[n]) * cd, av = absval(v[n]) * cd;
        f.gx[n] = gx;
        f.gy[n] = gy;
        if constexpr (PH) f.al[n] = al;
        f.u12[n] = u[n] * (C)(1.0 / 12.0);
        f.v12[n] = v[n] * (C)(1.0 / 12.0);
        f.au[n] = au;
        f.av[n] = av;
        f.c0[n] = c1 - (C)(2 * WSUM) * al - (C)6 * (au + av);
    }
}

// right-hand side L(Y) of eq. energy at both nodes of a slot with coefficients f, from the 6 x 5
// window of the stage input (rows[r]: column -2 of window row r, rows -2 .. 3 of the upper node)
template <typename C, bool PH>
__device__ __forceinline__ void thermal_rhs(const C *const rows[6], const Consts<C> &K, const ThCoef<C, PH> &f,
                                            bool phase, C k[2])
{
    RowQ<C> q[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) q[r] = row_q(rows[r]);
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const RowQ<C> *w = q + n;  // rows -2 .. 2 of node n
        const C y0 = w[2].h0;
        // sums and differences of the column's opposite neighbours
        const C S1 = w[3].h0 + w[1].h0, S2 = w[4].h0 + w[0].h0;
        const C D1 = w[3].h0 - w[1].h0, D2 = w[4].h0 - w[0].h0;
        // Laplacian without its centre term: 2 alpha sum_k w_k Y(x + e_k), by weight class
        const C l1 = w[2].s1 + S1, l4 = w[2].s2 + S2, l2 = w[3].s1 + w[1].s1;
        const C l5 = (w[3].s2 + w[1].s2) + (w[4].s1 + w[0].s1), l8 = w[4].s2 + w[0].s2;
        // (a run without phase-dependent properties takes the same arithmetic in either launch,
        // so batching it with runs that have them does not change its result)
        C lap;
        if (PH && phase)
            lap = f.al[PH ? n : 0] * ((C)(2 * W1) * l1 + (C)(2 * W4) * l4 + (C)(2 * W2) * l2 + (C)(2 * W5) * l5 +
                                      (C)(2 * W8) * l8);
        else
            lap = K.alpha2w1 * l1 + K.alpha2w4 * l4 + K.alpha2w2 * l2 + K.alpha2w5 * l5 + K.alpha2w8 * l8;
        // third-order upwind-biased convection without its centre term
        const C conv = f.u12[n] * ((C)8 * w[2].d1 - w[2].d2) + f.au[n] * (w[2].s2 - (C)4 * w[2].s1) +
                       f.v12[n] * ((C)8 * D1 - D2) + f.av[n] * (S2 - (C)4 * S1);
        // centre: Laplacian, convection and the linear part of the pressure-work source
        // T (c1 + c2 phi'(T)), phi'(T) = A / sqrt(T) + B
        k[n] = (lap - conv) + f.gx[n] * grad_x(w) + f.gy[n] * grad_y(w) + f.c0[n] * y0 + f.c2[n] * Ar<C>::sqrt_(y0);
    }
}

template <typename C, int TX, int TY, int NS, int NT, bool PH> struct Thermal {
    using G = ThGeom<TX, TY, NS>;
    static constexpr int H = G::H, RW = G::RW, RN = G::RN, NSLOT = G::NSLOT;
    static constexpr int ITER = (NSLOT + NT - 1) / NT;

    // Once the stage invariants are formed, rho holds every other stage input (and, with RK_IN_LDS,
    // ux the slots' T^n and uy their Runge-Kutta accumulators, by position)
    struct Smem {
        C Y[RN], rho[RN], ux[RN], uy[RN];
    };
    using Coef = ThCoef<C, PH>;
    // When a thread's last slot lies outside every stage after the first (the outer ring of a tile
    // with few threads), that slot forms its stage-1 k together with its invariants and keeps only
    // that, not its coefficients
    static constexpr bool LAST_S1 = ITER > 1 && G::count(2) <= NT * (ITER - 1);
    static constexpr int NCOEF = LAST_S1 ? ITER - 1 : ITER;
    // With many slots per thread, T^n and the accumulators of the slots' nodes live in LDS (in ux and
    // uy, free once the invariants are formed) rather than in registers; the arithmetic is the same
    static constexpr bool RK_IN_LDS = ITER >= 3;
    static constexpr int NRK = RK_IN_LDS ? 1 : ITER;
    // per-slot state, in registers
    struct Slots {
        // LDS position of the upper node (low 16 bits) and the one the operator is evaluated at
        // for it (high 16 bits; both nodes held: no evaluation)
        unsigned pos[ITER];
        __device__ int own(int j) const { return (int)(pos[j] & 0xffffu); }
        __device__ int ev(int j) const { return (int)(pos[j] >> 16); }
        __device__ bool evaluated(int j) const { return ((hold >> (2 * j)) & 3u) != 3u; }
        unsigned hold;   // bit 2 j + n: node n of slot j keeps its value (solid, inlet or wall ghost)
        Coef cf[NCOEF];
        C k1[2];         // LAST_S1: stage-1 k of the last slot
        C T0[NRK][2], acc[NRK][2];  // (!RK_IN_LDS)
    };

    // The frozen fields rho, u and T^n on the region of the tile at (rx0, ry0) (ghost columns per the
    // boundary conditions).  Every position of the thread: all loads are issued before the first LDS
    // write (one memory round trip); ghost positions map to valid nodes, so every load is in bounds,
    // and the ghost values replace the loaded ones afterwards.  INTERIOR: the region lies inside the
    // domain (direct indexing, no ghosts).
    template <bool INTERIOR>
    __device__ static void load_region(Smem &sm, const RunDev &R, const Consts<C> &K, int rx0, int ry0, int pt)
    {
        constexpr int RX = G::RX, RH = G::RH, IL = (RX * RH + NT - 1) / NT;
        const int P = R.pitch;
        C lr[IL], lu[IL], lv[IL], lt[IL];
        unsigned inlet = 0, wall = 0;
#pragma unroll
        for (int i = 0; i < IL; ++i) {
            const int n = min((int)threadIdx.x + NT * i, RX * RH - 1);
            const int lx = n % RX, ly = n / RX;
            int rx = rx0 + lx, ry = ry0 + ly;
            if constexpr (!INTERIOR) {
                const int kind = map_pos<PH>(R, rx0 + lx, ry0 + ly, rx, ry);
                if (kind == INLET_GHOST) inlet |= 1u << i;
                if (PH && kind == WALL_GHOST) wall |= 1u << i;
            }
            const unsigned idx = (unsigned)(ry * P + rx);
            lr[i] = ld_at<C>(R.rho, idx);
            lu[i] = ld_at<C>(R.ux, idx);
            lv[i] = ld_at<C>(R.uy, idx);
            lt[i] = ld_at<C>(R.T[pt], idx);
        }
#pragma unroll
        for (int i = 0; i < IL; ++i) {
            // (a thread past the region rewrites the last position with the value loaded for it,
            // so that no load is sunk behind a branch)
            const int n = min((int)threadIdx.x + NT * i, RX * RH - 1);
            const int p = (n / RX) * RW + n % RX;
            if constexpr (INTERIOR) {
                sm.rho[p] = lr[i];
                sm.ux[p] = lu[i];
                sm.uy[p] = lv[i];
                sm.Y[p] = lt[i];
            } else {
                const bool w = (wall >> i) & 1u;
                sm.rho[p] = w ? K.rho_w : lr[i];
                sm.ux[p] = w ? (C)0 : lu[i];
                sm.uy[p] = w ? (C)0 : lv[i];
                sm.Y[p] = ((inlet >> i) & 1u) ? K.T_sat : (w ? K.T_w : lt[i]);
            }
        }
    }

    // right-hand side L(Y) of eq. energy at both nodes of a slot with coefficients f, evaluated at
    // LDS positions c and c + RW of the stage input Y
    __device__ static void rhs(const C *Y, const Consts<C> &K, const Coef &f, int c, bool phase, C k[2])
    {
        // the 6 x 5 window read as positive offsets from its lowest corner
        const C *b = Y + opaque_index(c - 2 * RW - 2);
        const C *rows[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) rows[r] = b + r * RW;
        thermal_rhs<C, PH>(rows, K, f, phase, k);
    }

    // stage s: k = L(Y) on the slots of the tile grown by 2 (NS - s), then the next stage input.
    // The stage inputs alternate between two LDS arrays (Y and, once the stage invariants are
    // formed, the density's), so a slot writes its next input as soon as its k is known: one barrier
    // per stage.  CLEAN: a tile with no held position (inside the domain, away from the cylinder),
    // which skips the per-node hold test.
    template <int s, bool CLEAN>
    __device__ static void stage(Smem &sm, const Consts<C> &K, Slots &S, bool phase)
    {
        constexpr int CNT = G::count(s);
        const C *Yin = (s & 1) ? sm.Y : sm.rho;
        C *Yout = (s & 1) ? sm.rho : sm.Y;
#pragma unroll
        for (int j = 0; j < ITER; ++j) {
            const int r = threadIdx.x + NT * j;
            if (r >= CNT) continue;
            C kv[2] = {(C)0, (C)0};
            if (LAST_S1 && s == 1 && j == ITER - 1) { kv[0] = S.k1[0]; kv[1] = S.k1[1]; }
            else if (CLEAN || S.evaluated(j)) rhs(Yin, K, S.cf[j < NCOEF ? j : 0], S.ev(j), phase, kv);
#pragma unroll
            for (int n = 0; n < 2; ++n) {
                const int o = S.own(j) + n * RW;
                // a held node takes k = 0: the update then rewrites its value unchanged (in stage 1
                // that copies it into the second array), without a branch per node
                C k = kv[n];
                if constexpr (!CLEAN) k = ((S.hold >> (2 * j + n)) & 1u) ? (C)0 : k;
                const int jr = RK_IN_LDS ? 0 : j;
                C t0, a;
                if constexpr (s == 1) {
                    t0 = Yin[o];
                    if constexpr (RK_IN_LDS) sm.ux[o] = t0;
                    else S.T0[jr][n] = t0;
                } else {
                    t0 = RK_IN_LDS ? sm.ux[o] : S.T0[jr][n];
                    a = RK_IN_LDS ? sm.uy[o] : S.acc[jr][n];
                }
                if constexpr (NS == 4) {
                    if constexpr (s == 1) { a = k; Yout[o] = t0 + (C)0.5 * k; }
                    else if constexpr (s == 2) { a += (C)2 * k; Yout[o] = t0 + (C)0.5 * k; }
                    else if constexpr (s == 3) { a += (C)2 * k; Yout[o] = t0 + k; }
                    else { a = t0 + (a + k) * (C)(1.0 / 6.0); }
                } else {
                    if constexpr (s == 1) { a = k; Yout[o] = t0 + k; }
                    else { a = t0 + (C)0.5 * (a + k); }
                }
                if constexpr (RK_IN_LDS) sm.uy[o] = a;
                else S.acc[jr][n] = a;
            }
        }
        if constexpr (s < NS) __syncthreads();  // the next stage input is complete
    }
};

// OCC > 0: ask the compiler for at least OCC waves per SIMD (a register budget)
template <typename C, int TX, int TY, int NS, int NT, bool PH, int OCC = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1))) void k_thermal(
    const RunDev *__restrict__ runs, const Tile *__restrict__ tiles, int pt, long long step)
{
    static_assert(!is_dual<C>, "the tangent precision takes k_thermal_tan");
    using Th = Thermal<C, TX, TY, NS, NT, PH>;
    using G = typename Th::G;
    constexpr int H = G::H, RX = G::RX, RW = G::RW, RH = G::RH, TN = G::TN, NSLOT = G::NSLOT, TSLOT = G::TSLOT;
    constexpr int ITER = Th::ITER;
    __shared__ typename Th::Smem sm;

    const Tile t = tiles[blockIdx.x];
    const RunDev &R = runs[t.run];
    const int x0 = t.tx * TX, y0 = t.ty * TY;
    const int nx = R.nx, ny = R.ny, P = R.pitch;
    if (step < R.warmup || R.rk == 0) {
        // this run does not advance its temperature in this step: carry T over
        const gp<const C> Tin = gin<C>(R.T[pt]);
        const gp<C> Tout = gout<C>(R.T[pt ^ 1]);
        for (int q = threadIdx.x; q < TN; q += NT) {
            const int gx = x0 + q % TX, gy = y0 + q / TX;
            if (gx < nx && gy < ny) Tout[(size_t)gy * P + gx] = Tin[(size_t)gy * P + gx];
        }
        return;
    }
    const Consts<C> K(R);
    // a tile whose whole region lies inside the domain needs no ghost mapping, and one whose region
    // misses the cylinder's box no solid test (same positions and kinds, fewer instructions)
    const int rx0 = x0 - H, ry0 = y0 - H;
    const bool interior = rx0 >= 0 && rx0 + RX <= nx && ry0 >= 0 && ry0 + RH <= ny;
    const bool no_solid = R.cyl_r <= 0 || (interior && (rx0 + RX <= R.cyl_x - R.cyl_r || rx0 > R.cyl_x + R.cyl_r ||
                                                       ry0 + RH <= R.cyl_y - R.cyl_r || ry0 > R.cyl_y + R.cyl_r));

    // LDS positions of this thread's slots, fetched from the constant table first so that their
    // latency overlaps the field loads
    int spos[ITER];
#pragma unroll
    for (int j = 0; j < ITER; ++j) {
        const int r = threadIdx.x + NT * j;
        spos[j] = r < NSLOT ? (int)kSlots<TX, TY, NS>.pos[r] : 0;
    }

    // the frozen fields and T^n on the whole region (ghost columns per the boundary conditions)
    if (interior) Th::template load_region<true>(sm, R, K, rx0, ry0, pt);
    else Th::template load_region<false>(sm, R, K, rx0, ry0, pt);
    __syncthreads();

    // slots and their stage-invariant coefficients (thermal_coef)
    const C cd = R.upwind_kind == 1 ? (C)0.25 : (C)(1.0 / 12.0);
    const int out_c = (nx - 1) - (x0 - H);  // LDS column of the last domain column
    const bool phase = PH && R.phase_props;
    typename Th::Slots S;
    S.hold = 0;
    S.k1[0] = S.k1[1] = 0;
    // (a stage-1-only last slot first, while no other slot's coefficients occupy registers)
#pragma unroll
    for (int jj = 0; jj < ITER; ++jj) {
        const int j = Th::LAST_S1 ? (jj == 0 ? ITER - 1 : jj - 1) : jj;
        S.pos[j] = 0;
        const bool last_s1 = Th::LAST_S1 && j == ITER - 1;
        typename Th::Coef tmp;
        typename Th::Coef &f = last_s1 ? tmp : S.cf[j < Th::NCOEF ? j : 0];
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            f.gx[n] = f.gy[n] = f.c0[n] = f.c2[n] = 0;
            f.u12[n] = f.v12[n] = f.au[n] = f.av[n] = 0;
            f.al[PH ? n : 0] = 0;
        }
        const int r = threadIdx.x + NT * j;
        if (r >= NSLOT) continue;
        const int p = spos[j];
        const int lx = p % RW, ly = p / RW;
        int rx, ry;
        int kind = NODE;
        if (interior) { rx = rx0 + lx; ry = ry0 + ly; }
        else kind = map_pos<PH>(R, rx0 + lx, ry0 + ly, rx, ry);
        S.pos[j] = (unsigned)p;
        // the kind of a position depends on its column only, so both nodes of a slot share it
        if (kind == INLET_GHOST || kind == WALL_GHOST) {
            S.hold |= 3u << (2 * j);
            continue;
        }
        const int ry1 = ry + 1 == ny ? 0 : ry + 1;
        const unsigned hj = no_solid ? 0u : (solid_at(R, rx, ry) ? 1u : 0u) | (solid_at(R, rx, ry1) ? 2u : 0u);
        S.hold |= hj << (2 * j);
        if (hj == 3u) continue;
        // an outlet ghost evaluates the operator at the last column of its row
        const int c = kind == OUTLET_GHOST ? ly * RW + out_c : p;
        S.pos[j] |= (unsigned)c << 16;
        const int corner = opaque_index(c - 2 * RW - 2);
        const C *rr[6], *ru[6], *rv[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            rr[k] = sm.rho + corner + k * RW;
            ru[k] = sm.ux + corner + k * RW;
            rv[k] = sm.uy + corner + k * RW;
        }
        thermal_coef<C, PH>(R, K, rr, ru, rv, hj, cd, f);
        // (T^n, the stage-1 input, is not written before the barrier that follows)
        if (last_s1) {
            Th::rhs(sm.Y, K, tmp, c, phase, S.k1);
        }
    }

    __syncthreads();  // the density array is read by every slot's invariants before stage 1 reuses it
    if (interior && no_solid) {
        Th::template stage<1, true>(sm, K, S, phase);
        Th::template stage<2, true>(sm, K, S, phase);
        if constexpr (NS == 4) {
            Th::template stage<3, true>(sm, K, S, phase);
            Th::template stage<4, true>(sm, K, S, phase);
        }
    } else {
        Th::template stage<1, false>(sm, K, S, phase);
        Th::template stage<2, false>(sm, K, S, phase);
        if constexpr (NS == 4) {
            Th::template stage<3, false>(sm, K, S, phase);
            Th::template stage<4, false>(sm, K, S, phase);
        }
    }

    // the tile's slots come first
#pragma unroll
    for (int j = 0; j < ITER; ++j) {
        const int r = threadIdx.x + NT * j;
        if (NT * j >= TSLOT || r >= TSLOT) continue;
        const int gx = x0 + r % TX, gy = y0 + 2 * (r / TX);
        if (gx >= nx) continue;
#pragma unroll
        for (int n = 0; n < 2; ++n)
            if (gy + n < ny)
                *at<C>(R.T[pt ^ 1], (unsigned)((gy + n) * P + gx)) =
                    ((S.hold >> (2 * j + n)) & 1u) ? K.T_w
                                                   : (Th::RK_IN_LDS ? sm.uy[S.own(j) + n * RW] : S.acc[Th::RK_IN_LDS ? 0 : j][n]);
    }
}

// ------------------------------------------------------------------------------------------
// k_thermal_strip: the temperature step of a column strip, marching down a chunk of rows
// ------------------------------------------------------------------------------------------
// Lane l owns column x0 - 8 + l: the strip's W = NT - 16 columns and an 8-column halo on either
// side.  Iteration i brings rows 2i, 2i+1 of the frozen fields and T^n (counted from 2 NS rows above
// the chunk) into rings of 8 rows in LDS and issues the loads of the next two.  The stage-invariant
// coefficients and stage 1 of a pair of rows follow two rows behind the rows brought in, stage s + 1
// two rows behind stage s, so stage NS finishes the pair 2 NS rows behind them.  Stage s evaluates
// the chunk grown by 2 (NS - s) rows at either end and the strip grown by as many columns: the halo
// is paid on two sides of a long strip instead of all four sides of a tile.  A pair keeps its
// coefficients, T^n and Runge-Kutta accumulator in registers from its stage 1 to its stage NS (NS
// sets in rotation); the loop is unrolled by the rings' period of four pairs, which fixes every ring
// slot and register set at compile time.  The arithmetic of a position is k_thermal's (thermal_coef,
// thermal_rhs, the same Runge-Kutta updates), so the results are the same bit for bit.
template <int NS, int NT> struct ThStrip {
    static_assert(NS == 2 || NS == 4, "RK2 or RK4");
    static constexpr int HX = 8, W = NT - 2 * HX, HY = 2 * NS;
    static constexpr int NA = 3 + NS;  // rings: rho, u_x, u_y, then the NS stage inputs
    static constexpr int RS = 8 * NT;  // values of one ring
};

// (the tile entry: strip tx, the chunk's first row ty and its row count pad, a multiple of 8, so that
// the march takes a whole number of ring periods)
template <typename C, int NS, int NT, bool PH, int OCC = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1))) void k_thermal_strip(
    const RunDev *__restrict__ runs, const Tile *__restrict__ tiles, int pt, long long step)
{
    static_assert(!is_dual<C>, "the tangent precision takes k_thermal_tan");
    using G = ThStrip<NS, NT>;
    constexpr int HX = G::HX, W = G::W, HY = G::HY, RS = G::RS;
    // the rings, with two guard values at either end: the windows of the two outermost lanes on each
    // side, which lie outside every stage, reach two columns past their rows
    __shared__ C ring[G::NA * RS + 4];

    const Tile t = tiles[blockIdx.x];
    const RunDev &R = runs[t.run];
    const int x0 = t.tx * W, y0 = t.ty, CH = t.pad;
    const int NI = CH / 2 + 2 * NS;  // iterations, a multiple of 4
    const int nx = R.nx, ny = R.ny, P = R.pitch;
    const int lane = threadIdx.x;
    const int gx = x0 - HX + lane;
    if (step < R.warmup || R.rk == 0) {
        // this run does not advance its temperature in this step: carry T over
        if (lane >= HX && lane < NT - HX && gx < nx) {
            const gp<const C> Tin = gin<C>(R.T[pt]);
            const gp<C> Tout = gout<C>(R.T[pt ^ 1]);
            for (int y = y0; y < min(y0 + CH, ny); ++y) Tout[(size_t)y * P + gx] = Tin[(size_t)y * P + gx];
        }
        return;
    }
    const Consts<C> K(R);
    const C cd = R.upwind_kind == 1 ? (C)0.25 : (C)(1.0 / 12.0);
    const bool phase = PH && R.phase_props;

    // the lane's column: its kind, the domain column it reads and the lane the operator is evaluated
    // at (for an outlet ghost, the last domain column's); inlet and wall ghosts hold their values
    int rx, ry_unused;
    const int kind = map_pos<PH>(R, gx, 0, rx, ry_unused);
    const int ev = kind == OUTLET_GHOST ? (nx - 1) - (x0 - HX) : lane;
    const bool ghost = kind == INLET_GHOST || kind == WALL_GHOST;
    const bool inlet = kind == INLET_GHOST, wall = PH && kind == WALL_GHOST;
    // rows of the march; a chunk whose region lies inside the domain and misses the cylinder's box
    // needs no solid test
    const int ry0 = y0 - HY, ry1 = y0 + CH + HY;
    const bool no_solid =
        R.cyl_r <= 0 || (x0 - HX >= 0 && x0 + W + HX <= nx && ry0 >= 0 && ry1 <= ny &&
                         (x0 + W + HX <= R.cyl_x - R.cyl_r || x0 - HX > R.cyl_x + R.cyl_r ||
                          ry1 <= R.cyl_y - R.cyl_r || ry0 > R.cyl_y + R.cyl_r));

    C *const own = ring + 2 + lane;          // the lane's column of ring 0, row slot 0
    const C *const win = ring + ev;          // column -2 of the lane's windows, ring 0, row slot 0
    const gp<C> Tout = gout<C>(R.T[pt ^ 1]);

    // rows 2i, 2i+1 of the march, in flight between iterations
    C lr[2], lu[2], lv[2], lt[2];
    auto load = [&](int i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const unsigned idx = (unsigned)(wrap(ry0 + 2 * i + j, ny) * P + rx);
            lr[j] = ld_at<C>(R.rho, idx);
            lu[j] = ld_at<C>(R.ux, idx);
            lv[j] = ld_at<C>(R.uy, idx);
            lt[j] = ld_at<C>(R.T[pt], idx);
        }
    };
    // per pair in flight (set p & 3 for pair p): coefficients, T^n, accumulators, held nodes
    ThCoef<C, PH> cf[4];
    C T0[4][2], acc[4][2];
    unsigned hold[4];

    // the window rows -2 .. 3 of the pair starting at ring row slot `top` of ring a
    auto window = [&](int a, int top, const C *rows[6]) {
#pragma unroll
        for (int r = 0; r < 6; ++r) rows[r] = win + a * RS + ((top - 2 + r) & 7) * NT;
    };
    // k of stage s of the pair in set p whose rows start at slot `top` (held nodes: k = 0)
    auto stage_k = [&](int s, int p, int top, C k[2]) {
        const C *rows[6];
        window(2 + s, top, rows);
        thermal_rhs<C, PH>(rows, K, cf[p], phase, k);
#pragma unroll
        for (int n = 0; n < 2; ++n) k[n] = ((hold[p] >> n) & 1u) ? (C)0 : k[n];
    };
    auto store = [&](int p, int row) {
        if (lane < HX || lane >= NT - HX || gx >= nx) return;
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            const int gy = ry0 + row + n;
            if (gy < ny) Tout[(size_t)gy * P + gx] = ((hold[p] >> n) & 1u) ? K.T_w : acc[p][n];
        }
    };

    auto iteration = [&](auto UU, int m) {
        constexpr int U = decltype(UU)::value;
        const int i = 4 * m + U;
        // rows 2i, 2i+1 into ring slots 2U, 2U+1 (ghost values replace the loaded ones)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            C *o = own + (2 * U + j) * NT;
            o[0] = wall ? K.rho_w : lr[j];
            o[RS] = wall ? (C)0 : lu[j];
            o[2 * RS] = wall ? (C)0 : lv[j];
            o[3 * RS] = inlet ? K.T_sat : (wall ? K.T_w : lt[j]);
        }
        if (i + 1 < NI) load(i + 1);
        // the new temperatures of the pair that finished its last stage in the previous iteration,
        // stored only now: they follow the loads just issued, so the next iteration's wait for those
        // loads does not wait for these stores as well (the counter of outstanding vector memory
        // operations drains in issue order)
        if (i >= 2 * NS + 1) store((U + 3 - NS) & 3, 2 * (i - NS - 1));
        __syncthreads();
        // pair i - 1 (rows 2i-2, 2i-1 at slots 2U-2, 2U-1): its coefficients, then stage 1
        if (i >= 2) {
            constexpr int p = (U + 3) & 3, top = (2 * U - 2) & 7;
            unsigned hj = ghost ? 3u : 0u;
            if (!no_solid && !ghost) {
                const int ya = wrap(ry0 + 2 * i - 2, ny), yb = ya + 1 == ny ? 0 : ya + 1;
                hj = (solid_at(R, rx, ya) ? 1u : 0u) | (solid_at(R, rx, yb) ? 2u : 0u);
            }
            hold[p] = hj;
            const C *rr[6], *ru[6], *rv[6];
            window(0, top, rr);
            window(1, top, ru);
            window(2, top, rv);
            thermal_coef<C, PH>(R, K, rr, ru, rv, 0u, cd, cf[p]);
            C k[2];
            stage_k(1, p, top, k);
#pragma unroll
            for (int n = 0; n < 2; ++n) {
                const C t0 = own[3 * RS + ((top + n) & 7) * NT];
                T0[p][n] = t0;
                acc[p][n] = k[n];
                own[4 * RS + ((top + n) & 7) * NT] = NS == 4 ? t0 + (C)0.5 * k[n] : t0 + k[n];
            }
        }
        __syncthreads();
        // pair i - 2: stage 2
        if (i >= 4) {
            constexpr int p = (U + 2) & 3, top = (2 * U - 4) & 7;
            C k[2];
            stage_k(2, p, top, k);
#pragma unroll
            for (int n = 0; n < 2; ++n) {
                if constexpr (NS == 4) {
                    acc[p][n] += (C)2 * k[n];
                    own[5 * RS + ((top + n) & 7) * NT] = T0[p][n] + (C)0.5 * k[n];
                } else {
                    acc[p][n] = T0[p][n] + (C)0.5 * (acc[p][n] + k[n]);
                }
            }
        }
        if constexpr (NS == 4) {
            __syncthreads();
            // pair i - 3: stage 3
            if (i >= 6) {
                constexpr int p = (U + 1) & 3, top = (2 * U - 6) & 7;
                C k[2];
                stage_k(3, p, top, k);
#pragma unroll
                for (int n = 0; n < 2; ++n) {
                    acc[p][n] += (C)2 * k[n];
                    own[6 * RS + ((top + n) & 7) * NT] = T0[p][n] + k[n];
                }
            }
            __syncthreads();
            // pair i - 4: stage 4 and the new temperature
            if (i >= 8) {
                constexpr int p = U & 3, top = (2 * U - 8) & 7;
                C k[2];
                stage_k(4, p, top, k);
#pragma unroll
                for (int n = 0; n < 2; ++n) acc[p][n] = T0[p][n] + (acc[p][n] + k[n]) * (C)(1.0 / 6.0);
            }
        }
    };

    load(0);
    for (int m = 0; m < NI / 4; ++m) {
        iteration(std::integral_constant<int, 0>{}, m);
        iteration(std::integral_constant<int, 1>{}, m);
        iteration(std::integral_constant<int, 2>{}, m);
        iteration(std::integral_constant<int, 3>{}, m);
    }
    // the last pair (pair NI - 1 - NS, whose set is (NI - 1 - NS) mod 4 with NI a multiple of 4)
    store((3 - NS) & 3, 2 * (NI - 1 - NS));
}

#pragma clang fp contract(on)

// k_thermal_tan: the same temperature step in the tangent precision, one position per slot (the
// 40-byte values of a slot pair's windows would not fit the registers); slots, stages and the
// stencils' grouping by weight class as in k_thermal, with the opposite-neighbour differences of a
// single 5 x 5 window
template <int TX, int TY, int NS> struct ThGeomTan {
    static constexpr int H = 2 * NS;
    // region of RX x RH positions stored with an odd row stride RW (the ring slots of a wavefront
    // are short row pieces a stride apart, which an even stride would put on few LDS banks)
    static constexpr int RX = TX + 2 * H, RW = RX + 1, RH = TY + 2 * H, RN = RW * RH, TN = TX * TY;
    static constexpr int count(int s) { return (TX + 4 * (NS - s)) * (TY + 4 * (NS - s)); }
    static constexpr int NSLOT = count(1);
};

template <int TX, int TY, int NS> struct SlotTableTan {
    unsigned short pos[ThGeomTan<TX, TY, NS>::NSLOT];
};

template <int TX, int TY, int NS> constexpr SlotTableTan<TX, TY, NS> make_slots_tan()
{
    using G = ThGeomTan<TX, TY, NS>;
    SlotTableTan<TX, TY, NS> t{};
    int r = 0;
    for (int y = 0; y < TY; ++y)
        for (int x = 0; x < TX; ++x) t.pos[r++] = (unsigned short)((G::H + y) * G::RW + G::H + x);
    // ring k: the tile grown by 2k nodes minus the tile grown by 2(k - 1)
    for (int k = 1; k < NS; ++k) {
        const int o = G::H - 2 * k, A = TX + 4 * (k - 1), B = TY + 4 * (k - 1);
        for (int yy = 0; yy < 2; ++yy)
            for (int xx = 0; xx < A + 4; ++xx) t.pos[r++] = (unsigned short)((o + yy) * G::RW + o + xx);
        for (int yy = 0; yy < 2; ++yy)
            for (int xx = 0; xx < A + 4; ++xx) t.pos[r++] = (unsigned short)((o + B + 2 + yy) * G::RW + o + xx);
        for (int yy = 0; yy < B; ++yy)
            for (int q = 0; q < 4; ++q) t.pos[r++] = (unsigned short)((o + 2 + yy) * G::RW + o + (q < 2 ? q : A + q));
    }
    return t;
}

template <int TX, int TY, int NS> __constant__ const SlotTableTan<TX, TY, NS> kSlotsTan = make_slots_tan<TX, TY, NS>();

template <typename C, int TX, int TY, int NS, int NT, bool PH> struct ThermalTan {
    using G = ThGeomTan<TX, TY, NS>;
    static constexpr int H = G::H, RW = G::RW, RN = G::RN, TN = G::TN, NSLOT = G::NSLOT;
    static constexpr int ITER = (NSLOT + NT - 1) / NT;

    struct Smem {
        C Y[RN], rho[RN], ux[RN], uy[RN];
    };
    // per-slot state, in registers
    struct Slots {
        int own[ITER];  // LDS position of the slot
        int ev[ITER];   // LDS position the operator is evaluated at; < 0: value held (solid, inlet ghost)
        C T0[ITER], acc[ITER];
        // coefficients of L(Y) at the slot (8 registers, which keeps the occupancy of tiles with
        // many slots per thread): u/12, v/12 and |u| c_d, |v| c_d of the upwind convection, the
        // density-gradient coefficients gx, gy, the centre coefficient c0 (the Laplacian's and the
        // convection's centre weights and the linear part c1 of the source) and c2 of sqrt(Y)
        C u12[ITER], v12[ITER], au[ITER], av[ITER];
        C gx[ITER], gy[ITER], c0[ITER], c2[ITER];
        C al[PH ? ITER : 1];  // alpha at the slot (phase-dependent properties)
    };

    // right-hand side L(Y) of eq. energy at LDS position c with the coefficients of slot j
    __device__ static C rhs(const Smem &sm, const Consts<C> &K, const Slots &S, int j, int c, bool phase)
    {
        // the 5x5 window read as positive offsets from its lowest corner
        const C *b = sm.Y + opaque_index(c - 2 * RW - 2);
#define Y_(dx, dy) b[(2 + (dy)) * RW + 2 + (dx)]
        const C y0 = Y_(0, 0);
        // sums and differences of opposite neighbours
        const C p10 = Y_(1, 0), m10 = Y_(-1, 0), p20 = Y_(2, 0), m20 = Y_(-2, 0);
        const C p01 = Y_(0, 1), m01 = Y_(0, -1), p02 = Y_(0, 2), m02 = Y_(0, -2);
        const C S10 = p10 + m10, S20 = p20 + m20, S01 = p01 + m01, S02 = p02 + m02;
        PairD<C> d;
        d.d10 = p10 - m10; d.d20 = p20 - m20; d.d01 = p01 - m01; d.d02 = p02 - m02;
        const C a11 = Y_(1, 1), b11 = Y_(-1, -1), a1m = Y_(1, -1), b1m = Y_(-1, 1);
        const C a21 = Y_(2, 1), b21 = Y_(-2, -1), a2m = Y_(2, -1), b2m = Y_(-2, 1);
        const C a12 = Y_(1, 2), b12 = Y_(-1, -2), a1m2 = Y_(1, -2), b1m2 = Y_(-1, 2);
        const C a22 = Y_(2, 2), b22 = Y_(-2, -2), a2m2 = Y_(2, -2), b2m2 = Y_(-2, 2);
#undef Y_
        d.d11 = a11 - b11; d.d1m = a1m - b1m; d.d21 = a21 - b21; d.d2m = a2m - b2m;
        d.d12 = a12 - b12; d.d1m2 = a1m2 - b1m2; d.d22 = a22 - b22; d.d2m2 = a2m2 - b2m2;
        // axis pairs: Laplacian, upwind convection and the axis part of the gradient term
        const C a = (PH && phase) ? S.al[PH ? j : 0] : K.alpha;
        const C ax = (C)(2 * W1) * a * (S10 + S01) + (C)(2 * W4) * a * (S20 + S02) -
                     (S.u12[j] * ((C)8 * d.d10 - d.d20) + S.au[j] * (S20 - (C)4 * S10) +
                      S.v12[j] * ((C)8 * d.d01 - d.d02) + S.av[j] * (S02 - (C)4 * S01)) +
                     S.gx[j] * ((C)W1 * d.d10 + (C)(2 * W4) * d.d20) +
                     S.gy[j] * ((C)W1 * d.d01 + (C)(2 * W4) * d.d02);
        // diagonal pairs: Laplacian (2 alpha w_k) and the diagonal part of the gradient term
        const C s2 = (a11 + b11) + (a1m + b1m);
        const C s5 = ((a21 + b21) + (a2m + b2m)) + ((a12 + b12) + (a1m2 + b1m2));
        const C s8 = (a22 + b22) + (a2m2 + b2m2);
        C dg;
        // (a run without phase-dependent properties takes the same arithmetic in either launch, so
        // batching it with runs that have them does not change its result)
        if (PH && phase)
            dg = S.al[PH ? j : 0] * ((C)(2 * W2) * s2 + (C)(2 * W5) * s5 + (C)(2 * W8) * s8);
        else
            dg = K.alpha2w2 * s2 + K.alpha2w5 * s5 + K.alpha2w8 * s8;
        const C gdx = (C)W2 * (d.d11 + d.d1m) + (C)W5 * ((C)2 * (d.d21 + d.d2m) + d.d12 + d.d1m2) +
                      (C)(2 * W8) * (d.d22 + d.d2m2);
        const C gdy = (C)W2 * (d.d11 - d.d1m) + (C)W5 * (d.d21 - d.d2m + (C)2 * (d.d12 - d.d1m2)) +
                      (C)(2 * W8) * (d.d22 - d.d2m2);
        // centre: Laplacian, convection and the linear part of the pressure-work source
        // T (c1 + c2 phi'(T)), phi'(T) = A / sqrt(T) + B
        return ax + dg + S.gx[j] * gdx + S.gy[j] * gdy + S.c0[j] * y0 + S.c2[j] * Ar<C>::sqrt_(y0);
    }

    // stage s: k = L(Y) on the slots of the tile grown by 2 (NS - s), then the next stage input
    template <int s>
    __device__ static void stage(Smem &sm, const Consts<C> &K, Slots &S, bool phase)
    {
        constexpr int CNT = G::count(s);
        C kv[ITER];
#pragma unroll
        for (int j = 0; j < ITER; ++j) {
            kv[j] = 0;
            const int r = threadIdx.x + NT * j;
            if (r >= CNT || S.ev[j] < 0) continue;
            kv[j] = rhs(sm, K, S, j, S.ev[j], phase);
        }
        if constexpr (s < NS) __syncthreads();  // every stage input has been read
#pragma unroll
        for (int j = 0; j < ITER; ++j) {
            const int r = threadIdx.x + NT * j;
            if (r >= CNT || S.ev[j] < 0) continue;
            const C k = kv[j];
            const int o = S.own[j];
            if constexpr (NS == 4) {
                if constexpr (s == 1) { S.acc[j] = k; sm.Y[o] = S.T0[j] + (C)0.5 * k; }
                else if constexpr (s == 2) { S.acc[j] += (C)2 * k; sm.Y[o] = S.T0[j] + (C)0.5 * k; }
                else if constexpr (s == 3) { S.acc[j] += (C)2 * k; sm.Y[o] = S.T0[j] + k; }
                else { S.acc[j] = S.T0[j] + (S.acc[j] + k) * (C)(1.0 / 6.0); }
            } else {
                if constexpr (s == 1) { S.acc[j] = k; sm.Y[o] = S.T0[j] + k; }
                else { S.acc[j] = S.T0[j] + (C)0.5 * (S.acc[j] + k); }
            }
        }
        if constexpr (s < NS) __syncthreads();
    }
};

template <typename C, int TX, int TY, int NS, int NT, bool PH>
__global__ __launch_bounds__(NT) void k_thermal_tan(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles, int pt,
                                                long long step)
{
    using Th = ThermalTan<C, TX, TY, NS, NT, PH>;
    constexpr int H = Th::H, RX = Th::G::RX, RW = Th::RW, RH = Th::G::RH, TN = Th::TN, NSLOT = Th::NSLOT;
    constexpr int ITER = Th::ITER;
    __shared__ typename Th::Smem sm;

    const Tile t = tiles[blockIdx.x];
    const RunDev &R = runs[t.run];
    const int x0 = t.tx * TX, y0 = t.ty * TY;
    const int nx = R.nx, ny = R.ny, P = R.pitch;
    if (step < R.warmup || R.rk == 0) {
        // this run does not advance its temperature in this step: carry T over
        const gp<const C> Tin = gin<C>(R.T[pt]);
        const gp<C> Tout = gout<C>(R.T[pt ^ 1]);
        for (int q = threadIdx.x; q < TN; q += NT) {
            const int gx = x0 + q % TX, gy = y0 + q / TX;
            if (gx < nx && gy < ny) Tout[(size_t)gy * P + gx] = Tin[(size_t)gy * P + gx];
        }
        return;
    }
    const Consts<C> K(R);

    // LDS positions of this thread's slots, fetched from the constant table first so that their
    // latency overlaps the field loads
    int spos[ITER];
#pragma unroll
    for (int j = 0; j < ITER; ++j) {
        const int r = threadIdx.x + NT * j;
        spos[j] = r < NSLOT ? (int)kSlotsTan<TX, TY, NS>.pos[r] : 0;
    }

    // the frozen fields and T^n on the whole region (ghost columns per the boundary conditions)
    {
        // (40-byte values: one position at a time keeps the registers low)
        for (int n = threadIdx.x; n < RX * RH; n += NT) {
            const int lx = n % RX, ly = n / RX, p = ly * RW + lx;
            int rx, ry;
            const int kind = map_pos<PH>(R, x0 - H + lx, y0 - H + ly, rx, ry);
            const unsigned idx = (unsigned)(ry * P + rx);
            sm.rho[p] = ld_at<C>(R.rho, idx);
            sm.ux[p] = ld_at<C>(R.ux, idx);
            sm.uy[p] = ld_at<C>(R.uy, idx);
            sm.Y[p] = kind == INLET_GHOST ? K.T_sat : ld_at<C>(R.T[pt], idx);
        }
    }
    __syncthreads();

    // slots and their stage-invariant coefficients:
    //   gx, gy = alpha grad(rho)/rho;  source(T) = c1 T + c2 sqrt(T) with
    //   D = div(u)/(rho cv), c1 = -D R rho/(1 - b rho) + B D a rho^2/(1 + 2 b rho - b^2 rho^2),
    //   c2 = A D a rho^2/(1 + 2 b rho - b^2 rho^2), phi'(T) = A/sqrt(T) + B
    const C cd = R.upwind_kind == 1 ? (C)0.25 : (C)(1.0 / 12.0);
    const int out_c = (nx - 1) - (x0 - H);  // LDS column of the last domain column
    typename Th::Slots S;
#pragma unroll
    for (int j = 0; j < ITER; ++j) {
        S.own[j] = 0; S.ev[j] = -1;
        S.T0[j] = S.acc[j] = S.gx[j] = S.gy[j] = S.c0[j] = S.c2[j] = 0;
        if constexpr (PH) S.al[j] = 0;
        S.u12[j] = S.v12[j] = S.au[j] = S.av[j] = 0;
        const int r = threadIdx.x + NT * j;
        if (r >= NSLOT) continue;
        const int p = spos[j];
        const int lx = p % RW, ly = p / RW;
        int rx, ry;
        const int kind = map_pos<PH>(R, x0 - H + lx, y0 - H + ly, rx, ry);
        S.own[j] = p;
        S.T0[j] = sm.Y[p];
        if (kind == INLET_GHOST || kind == WALL_GHOST || solid_at(R, rx, ry)) continue;
        // an outlet ghost evaluates the operator at the last column of its row
        const int c = kind == OUTLET_GHOST ? ly * RW + out_c : p;
        S.ev[j] = c;
        const PairD<C> dr = pair_diffs<RW>(sm.rho, c);
        const PairD<C> du = pair_diffs<RW>(sm.ux, c);
        const PairD<C> dv = pair_diffs<RW>(sm.uy, c);
        const C rho = sm.rho[c];
        const C ir = Ar<C>::rcp(rho);
        // (1/(rho cv)) div(lambda grad T) with lambda = rho cv alpha(rho):
        //   alpha (lap T + grad rho . grad T / rho) + alpha'(rho) grad rho . grad T
        C dal;
        const C al = alpha_at<PH>(R, K, rho, dal);
        const C gcoef = al * ir + dal;
        const C gx = gcoef * dr.gx();
        const C gy = gcoef * dr.gy();
        const C D = (du.gx() + dv.gy()) * ir * K.inv_cv;
        const C d1 = (C)1 - K.b * rho;
        const C d2 = (C)1 + (C)2 * K.b * rho - K.b * K.b * rho * rho;
        const C A2 = D * K.a * rho * rho * Ar<C>::rcp(d2);
        const C c1 = -D * rho * K.Rg * Ar<C>::rcp(d1) + K.dphi_B * A2;
        S.c2[j] = K.dphi_A * A2;
        // third-order upwind-biased convection per axis:
        //   u (8 d1 - d2) / 12 + |u| c_d (S2 - 4 S1 + 6 Y)   (d, S: differences / sums of the pair)
        const C u = sm.ux[c], v = sm.uy[c];
        const C au = absval(u) * cd, av = absval(v) * cd;
        const C u12 = u * (C)(1.0 / 12.0), v12 = v * (C)(1.0 / 12.0);
        S.gx[j] = gx;
        S.gy[j] = gy;
        if constexpr (PH) S.al[j] = al;
        S.u12[j] = u12;
        S.v12[j] = v12;
        S.au[j] = au;
        S.av[j] = av;
        S.c0[j] = c1 - (C)(2 * WSUM) * al - (C)6 * (au + av);
    }

    const bool phase = PH && R.phase_props;
    Th::template stage<1>(sm, K, S, phase);
    Th::template stage<2>(sm, K, S, phase);
    if constexpr (NS == 4) {
        Th::template stage<3>(sm, K, S, phase);
        Th::template stage<4>(sm, K, S, phase);
    }

    // the tile's slots come first
#pragma unroll
    for (int j = 0; j < ITER; ++j) {
        const int r = threadIdx.x + NT * j;
        if (NT * j >= TN || r >= TN) continue;
        const int gx = x0 + r % TX, gy = y0 + r / TX;
        if (gx >= nx || gy >= ny) continue;
        *at<C>(R.T[pt ^ 1], (unsigned)(gy * P + gx)) = S.ev[j] < 0 ? K.T_w : S.acc[j];
    }
}


// ------------------------------------------------------------------------------------------
// Diagnostics: FP64 mass and wall heat flux (Sec. IV B), one launch for all runs whose sample falls
// on this step, fixed reduction order (bitwise reproducible)
// ------------------------------------------------------------------------------------------
template <typename A> __device__ inline double val(const A &x) { return (double)x; }
template <typename A> __device__ inline double der(const A &, int) { return 0.0; }
template <> __device__ inline double der<Dual>(const Dual &x, int k) { return x.d[k]; }

// thermal diffusivity of the vapour (lambda_v = rho_v c_v alpha_v normalises Nu)
template <typename A> __device__ inline A vapour_alpha(const RunDev &R, const Consts<A> &K)
{
    return R.phase_props ? (A)R.alpha_v : K.alpha;
}

// sum over the 256 threads of a workgroup in a fixed order: FP64 values across each wavefront by
// butterfly shuffles, then the four wavefronts' sums in LDS; tangent values by an LDS tree
template <typename A> __device__ inline A block_sum(A v, A *lds)
{
    if constexpr (std::is_same<A, double>::value) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
        __syncthreads();
        const A s = (lds[0] + lds[1]) + (lds[2] + lds[3]);
        __syncthreads();
        return s;
    } else {
        lds[threadIdx.x] = v;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) lds[threadIdx.x] = lds[threadIdx.x] + lds[threadIdx.x + w];
            __syncthreads();
        }
        const A s = lds[0];
        __syncthreads();
        return s;
    }
}

// Whether a run's diagnostic takes part in a launch: a read-out of run `readout` (>= 0), or the
// run's Nu sample (acc) or finiteness check falling on `step`.
__device__ inline bool diag_fires(const RunDev &R, int run, long long step, int readout, bool &acc)
{
    acc = readout < 0 && R.diag_every > 0 && step >= R.warmup && step % R.diag_every == 0;
    const bool chk = readout < 0 && R.check_every > 0 && step % R.check_every == 0;
    return readout >= 0 ? run == readout : (acc || chk);
}

// partial FP64 sums of the density over the rows of each diagnostic workgroup (fluid nodes, row by
// row, the cylinder's rows with the solid test)
template <typename C>
__global__ __launch_bounds__(256) void k_diag_partial(const RunDev *__restrict__ runs, const DiagBlock *__restrict__ blocks,
                                                      long long step, int readout)
{
    const DiagBlock b = blocks[blockIdx.x];
    const RunDev &R = runs[b.run];
    bool acc;
    if (!diag_fires(R, b.run, step, readout, acc)) return;
    __shared__ double lds[4];
    const gp<const C> rho = gin<C>(R.rho);
    double s = 0.0;
    const int r2 = R.cyl_r * R.cyl_r;
    constexpr int V = std::is_same<C, float>::value ? 4 : (std::is_same<C, double>::value ? 2 : 1);
    if constexpr (V > 1) {
        // 16 bytes (V values) per lane and load, eight loads in flight before they are summed; the
        // workgroup's rows are contiguous (pitch apart, the pitch a multiple of 64 values, every row
        // 256-byte aligned), so chunk q of them is row q / nc, columns V (q % nc) on; a chunk past the
        // last one is loaded clamped and not taken
        typedef C Vec __attribute__((ext_vector_type(V)));
        constexpr int U = 8;
        const int nc = R.pitch / V, nq = (b.row1 - b.row0) * nc;
        const gp<const Vec> base = (gp<const Vec>)(rho + (size_t)b.row0 * R.pitch);
        for (int q0 = threadIdx.x; q0 < nq; q0 += 256 * U) {
            Vec v[U];
#pragma unroll
            for (int j = 0; j < U; ++j) v[j] = base[min(q0 + 256 * j, nq - 1)];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int q = q0 + 256 * j, yr = q / nc, dy = b.row0 + yr - R.cyl_y;
                const bool in = q < nq, cut = (R.cyl_r > 0) & (dy * dy <= r2);
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    // the conditions are combined without short-circuit branches, into one select (the
                    // branched form lost the value of a taken node next to the cylinder in the FP64
                    // instantiation built by hipcc 7.2 for gfx950)
                    const int x = V * (q - yr * nc) + e, dx = x - R.cyl_x;
                    const bool take = in & (x < R.nx) & !(cut & (dx * dx + dy * dy <= r2));
                    s += take ? (double)v[j][e] : 0.0;
                }
            }
        }
        s = block_sum<double>(s, lds);
        if (threadIdx.x == 0) R.partials[b.index] = s;
        return;
    }
    // four row positions per thread and pass, loaded before they are summed (their loads overlap)
    for (int y = b.row0; y < b.row1; ++y) {
        const gp<const C> row = rho + (size_t)y * R.pitch;
        const int dy = y - R.cyl_y;
        const bool cut = R.cyl_r > 0 && dy * dy <= r2;
        for (int x0 = threadIdx.x; x0 < R.nx; x0 += 1024) {
            C v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int x = min(x0 + 256 * j, R.nx - 1);
                v[j] = row[x];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int x = x0 + 256 * j, dx = x - R.cyl_x;
                const bool take = x < R.nx && !(cut && dx * dx + dy * dy <= r2);
                s += take ? (double)v[j] : 0.0;
            }
        }
    }
    s = block_sum<double>(s, lds);
    if (threadIdx.x == 0) R.partials[b.index] = s;
}

// one workgroup per run: the partial sums in their fixed order, the wall probes (q_p, Nu), the
// accumulators
template <typename C>
__global__ __launch_bounds__(256) void k_diag_final(const RunDev *__restrict__ runs, int run0, int pt, long long step,
                                                    int readout)
{
    using A = typename std::conditional<is_dual<C>, Dual, double>::type;
    const int run = run0 + blockIdx.x;
    const RunDev &R = runs[run];
    bool acc;
    if (!diag_fires(R, run, step, readout, acc)) return;
    __shared__ A lds[is_dual<C> ? 256 : 4];
    __shared__ double ldsd[4];
    double m = 0.0;
    for (int k = threadIdx.x; k < R.nblk; k += 256) m += R.partials[k];
    const double mass = block_sum<double>(m, ldsd);
    const Consts<A> K(R);
    const gp<const C> rho = gin<C>(R.rho);
    const gp<const C> T = gin<C>(R.T[pt]);
    A qs = 0.0;
    for (int k = threadIdx.x; k < R.np; k += 256) {
        const double px = R.probes[2 * k], py = R.probes[2 * k + 1];
        const int x0 = (int)floor(px), y0 = (int)floor(py);
        const double fx = px - x0, fy = py - y0;
        const size_t i00 = (size_t)y0 * R.pitch + x0, i01 = i00 + R.pitch;
        const A w00 = (1 - fx) * (1 - fy), w10 = fx * (1 - fy), w01 = (1 - fx) * fy, w11 = fx * fy;
        const A r = w00 * (A)rho[i00] + w10 * (A)rho[i00 + 1] + w01 * (A)rho[i01] + w11 * (A)rho[i01 + 1];
        const A tp = w00 * (A)T[i00] + w10 * (A)T[i00 + 1] + w01 * (A)T[i01] + w11 * (A)T[i01 + 1];
        A dal;
        qs = qs + r * (A)R.cv * alpha_at<!is_dual<C>>(R, K, r, dal) * (K.T_w - tp) / (A)1.5;
    }
    A q = block_sum<A>(qs, lds);
    if (threadIdx.x == 0) {
        q = R.np > 0 ? q / (A)(double)R.np : (A)0.0;
        const A dT = K.T_w - K.T_sat;
        const A nu = (R.np > 0 && val(dT) != 0.0)
                         ? q * (A)2.0 * (A)(double)R.cyl_r / ((A)R.rho_v * (A)R.cv * vapour_alpha(R, K) * dT)
                         : (A)0.0;
        R.acc[0] = mass;
        R.acc[1] = val(q);
        R.acc[2] = val(nu);
        for (int k = 0; k < kTangents; ++k) R.acc[8 + k] = der(nu, k);
        if (acc) {
            R.acc[3] += val(nu);
            R.acc[4] += 1.0;
            for (int k = 0; k < kTangents; ++k) R.acc[12 + k] += der(nu, k);
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
    RawT<S> *f = (RawT<S> *)R.f[0];
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
// Launch variants (tile shape, threads per block) and launchers
// ------------------------------------------------------------------------------------------
// stream+collide: FP32 and reduced-precision storage / FP64
static const Variant kLbm32[] = {{32, 16, 256, 0}, {64, 16, 512, 0}, {32, 32, 512, 0}, {32, 8, 256, 0},
                                 {32, 8, 256, 6},  {64, 8, 512, 6},  {64, 8, 512, 7},
                                 // strips (k_lbm_strip): NT - 4 columns by a chunk of rows
                                 {124, 64, 128, 0}, {252, 32, 256, 0}, {60, 32, 64, 0}, {60, 64, 64, 0}};
static const Variant kLbm64[] = {{32, 16, 256, 0}, {16, 16, 256, 0}};
// temperature update (LDS holds 4 fields of the tile grown by 2 nodes per stage); 64 x 32 with 512
// threads also with a register budget of 4 waves per SIMD, which gives it a second workgroup per CU
static const Variant kTh32[] = {{64, 32, 512, 0}, {32, 32, 512, 0}, {64, 32, 1024, 0}, {32, 32, 256, 0},
                                {64, 32, 512, 4},
                                // strips of NT - 16 columns marching down chunks of rows: 64 rows, and
                                // chunks that spread the strips over the resident workgroups
                                {240, 64, 256, 2, 1}, {240, 0, 256, 2, 1}, {112, 0, 128, 2, 1}};
static const Variant kTh64[] = {{16, 16, 256, 0}, {32, 16, 256, 0}, {112, 64, 128, 2, 1}, {112, 0, 128, 2, 1}};
// tangent precision (40-byte values): one small tile each (the RK4 temperature tile with its
// 8-node halo stays within the 160 KB of LDS)
static const Variant kTanLbm[] = {{16, 16, 256, 0}};
static const Variant kTanTh[] = {{16, 8, 256, 0}};

int variant_count(int precision, int kernel)
{
    if (precision == 4) return 1;
    if (kernel == 0) return precision == 0 ? 2 : 11;
    return precision == 0 ? 4 : 8;
}


Variant variant_shape(int precision, int kernel, int v)
{
    if (v < 0 || v >= variant_count(precision, kernel)) return Variant{0, 0, 0, 0, 0};
    if (precision == 4) return kernel == 0 ? kTanLbm[v] : kTanTh[v];
    if (kernel == 0) return precision == 0 ? kLbm64[v] : kLbm32[v];
    return precision == 0 ? kTh64[v] : kTh32[v];
}

// Launch of a stencil kernel; with `tm`, through hipExtLaunchKernelGGL, whose start / stop events
// take the timestamps of the kernel's own dispatch (its duration inside the step sequence)
template <typename... P, typename... A>
static void dispatch(void (*kern)(P...), int grid, int block, hipStream_t st, const Timing *tm, A... args)
{
    if (tm) hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, tm->start, tm->stop, 0, static_cast<P>(args)...);
    else hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, static_cast<P>(args)...);
}

template <typename S, int TX, int TY, int NT, int OCC = 0>
static hipError_t lbm_go(bool write_f, bool phase, const RunDev *runs, const Tile *tiles, int n, int pf, int pt,
                         int ph, long long step, hipStream_t st, const Timing *tm)
{
    // phase-dependent properties are instantiated for FP32 and FP64 only
    constexpr bool kPhase = std::is_same<S, float>::value || std::is_same<S, double>::value;
    if constexpr (kPhase) {
        if (phase) {
            if (write_f) dispatch(k_lbm<S, TX, TY, NT, true, true, OCC>, n, NT, st, tm, runs, tiles, pf, pt, ph, step);
            else dispatch(k_lbm<S, TX, TY, NT, false, true, OCC>, n, NT, st, tm, runs, tiles, pf, pt, ph, step);
            return hipGetLastError();
        }
    } else {
        if (phase) return hipErrorInvalidValue;
    }
    if (write_f) dispatch(k_lbm<S, TX, TY, NT, true, false, OCC>, n, NT, st, tm, runs, tiles, pf, pt, ph, step);
    else dispatch(k_lbm<S, TX, TY, NT, false, false, OCC>, n, NT, st, tm, runs, tiles, pf, pt, ph, step);
    return hipGetLastError();
}

template <typename S, int NT, int CH, int OCC = 0>
static hipError_t strip_go(bool write_f, bool phase, const RunDev *runs, const Tile *tiles, int n, int pf, int pt,
                           int ph, long long step, hipStream_t st, const Timing *tm)
{
    constexpr bool kPhase = std::is_same<S, float>::value || std::is_same<S, double>::value;
    if constexpr (kPhase) {
        if (phase) {
            if (write_f) dispatch(k_lbm_strip<S, NT, CH, true, true, OCC>, n, NT, st, tm, runs, tiles, pf, pt, ph, step);
            else dispatch(k_lbm_strip<S, NT, CH, false, true, OCC>, n, NT, st, tm, runs, tiles, pf, pt, ph, step);
            return hipGetLastError();
        }
    } else {
        if (phase) return hipErrorInvalidValue;
    }
    if (write_f) dispatch(k_lbm_strip<S, NT, CH, true, false, OCC>, n, NT, st, tm, runs, tiles, pf, pt, ph, step);
    else dispatch(k_lbm_strip<S, NT, CH, false, false, OCC>, n, NT, st, tm, runs, tiles, pf, pt, ph, step);
    return hipGetLastError();
}

template <typename S>
static hipError_t lbm_impl(int v, bool write_f, bool phase, const RunDev *runs, const Tile *tiles, int n, int pf,
                           int pt, int ph, long long step, hipStream_t st, const Timing *tm)
{
    if (n <= 0) return hipSuccess;
    if constexpr (std::is_same<S, Dual>::value) {
        if (v != 0) return hipErrorInvalidValue;
        return lbm_go<S, 16, 16, 256>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
    } else if constexpr (std::is_same<S, double>::value) {
        switch (v) {
        case 0: return lbm_go<S, 32, 16, 256>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        case 1: return lbm_go<S, 16, 16, 256>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (v) {
        case 0: return lbm_go<S, 32, 16, 256>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        case 1: return lbm_go<S, 64, 16, 512>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        case 2: return lbm_go<S, 32, 32, 512>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        case 3: return lbm_go<S, 32, 8, 256>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        case 4: return lbm_go<S, 32, 8, 256, 6>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        case 5: return lbm_go<S, 64, 8, 512, 6>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        case 6: return lbm_go<S, 64, 8, 512, 7>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        case 7: return strip_go<S, 128, 64>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        case 8: return strip_go<S, 256, 32>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        case 9: return strip_go<S, 64, 32>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        case 10: return strip_go<S, 64, 64>(write_f, phase, runs, tiles, n, pf, pt, ph, step, st, tm);
        default: return hipErrorInvalidValue;
        }
    }
}

hipError_t launch_lbm(int precision, int variant, bool write_f, bool phase, const RunDev *runs_dev, const Tile *tiles,
                      int n_tiles, int pf, int pt, int ph, long long step, hipStream_t stream, const Timing *timing)
{
    switch (precision) {
    case 0: return lbm_impl<double>(variant, write_f, phase, runs_dev, tiles, n_tiles, pf, pt, ph, step, stream, timing);
    case 1: return lbm_impl<float>(variant, write_f, phase, runs_dev, tiles, n_tiles, pf, pt, ph, step, stream, timing);
    case 2: return lbm_impl<__half>(variant, write_f, phase, runs_dev, tiles, n_tiles, pf, pt, ph, step, stream, timing);
    case 3: return lbm_impl<__hip_bfloat16>(variant, write_f, phase, runs_dev, tiles, n_tiles, pf, pt, ph, step, stream, timing);
    case 4: return lbm_impl<Dual>(variant, write_f, phase, runs_dev, tiles, n_tiles, pf, pt, ph, step, stream, timing);
    default: return hipErrorInvalidValue;
    }
}

template <typename C, int TX, int TY, int NT, int OCC = 0>
static hipError_t th_go(int rk, bool phase, const RunDev *runs, const Tile *tiles, int n, int pt, long long step,
                        hipStream_t st, const Timing *tm)
{
    if constexpr (!is_dual<C>) {
        if (phase) {
            if (rk == 4) dispatch(k_thermal<C, TX, TY, 4, NT, true, OCC>, n, NT, st, tm, runs, tiles, pt, step);
            else if (rk == 2) dispatch(k_thermal<C, TX, TY, 2, NT, true, OCC>, n, NT, st, tm, runs, tiles, pt, step);
            else return hipErrorInvalidValue;
            return hipGetLastError();
        }
    } else {
        if (phase) return hipErrorInvalidValue;
    }
    if constexpr (is_dual<C>) {
        if (rk == 4) dispatch(k_thermal_tan<C, TX, TY, 4, NT, false>, n, NT, st, tm, runs, tiles, pt, step);
        else if (rk == 2) dispatch(k_thermal_tan<C, TX, TY, 2, NT, false>, n, NT, st, tm, runs, tiles, pt, step);
        else return hipErrorInvalidValue;
    } else {
        if (rk == 4) dispatch(k_thermal<C, TX, TY, 4, NT, false, OCC>, n, NT, st, tm, runs, tiles, pt, step);
        else if (rk == 2) dispatch(k_thermal<C, TX, TY, 2, NT, false, OCC>, n, NT, st, tm, runs, tiles, pt, step);
        else return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// the strip kernel of an RK order and launch kind
template <typename C, int NT, int OCC>
static const void *th_strip_fn(int rk, bool phase)
{
    if (phase) {
        if (rk == 4) return (const void *)k_thermal_strip<C, 4, NT, true, OCC>;
        if (rk == 2) return (const void *)k_thermal_strip<C, 2, NT, true, OCC>;
    } else {
        if (rk == 4) return (const void *)k_thermal_strip<C, 4, NT, false, OCC>;
        if (rk == 2) return (const void *)k_thermal_strip<C, 2, NT, false, OCC>;
    }
    return nullptr;
}

template <typename C, int NT, int OCC = 0>
static hipError_t th_strip_go(int rk, bool phase, const RunDev *runs, const Tile *tiles, int n, int pt, long long step,
                              hipStream_t st, const Timing *tm)
{
    static_assert(!is_dual<C>, "strips are built for the plain precisions");
    if (phase) {
        if (rk == 4) dispatch(k_thermal_strip<C, 4, NT, true, OCC>, n, NT, st, tm, runs, tiles, pt, step);
        else if (rk == 2) dispatch(k_thermal_strip<C, 2, NT, true, OCC>, n, NT, st, tm, runs, tiles, pt, step);
        else return hipErrorInvalidValue;
    } else {
        if (rk == 4) dispatch(k_thermal_strip<C, 4, NT, false, OCC>, n, NT, st, tm, runs, tiles, pt, step);
        else if (rk == 2) dispatch(k_thermal_strip<C, 2, NT, false, OCC>, n, NT, st, tm, runs, tiles, pt, step);
        else return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_thermal(int precision, int rk, int variant, bool phase, const RunDev *runs_dev, const Tile *tiles,
                          int n_tiles, int pt, long long step, hipStream_t stream, const Timing *timing)
{
    if (n_tiles <= 0) return hipSuccess;
    if (precision == 4) {
        if (variant != 0) return hipErrorInvalidValue;
        return th_go<Dual, 16, 8, 256>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
    }
    if (precision == 0) {
        switch (variant) {
        case 0: return th_go<double, 16, 16, 256>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
        case 1: return th_go<double, 32, 16, 256>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
        case 2: return th_strip_go<double, 128, 2>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
        case 3: return th_strip_go<double, 128, 2>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
        default: return hipErrorInvalidValue;
        }
    }
    switch (variant) {
    case 0: return th_go<float, 64, 32, 512>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
    case 1: return th_go<float, 32, 32, 512>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
    case 2: return th_go<float, 64, 32, 1024>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
    case 3: return th_go<float, 32, 32, 256>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
    case 4: return th_go<float, 64, 32, 512, 4>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
    case 5: return th_strip_go<float, 256, 2>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
    case 6: return th_strip_go<float, 256, 2>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
    case 7: return th_strip_go<float, 128, 2>(rk, phase, runs_dev, tiles, n_tiles, pt, step, stream, timing);
    default: return hipErrorInvalidValue;
    }
}

int chunked_blocks_per_cu(int precision, int variant, int rk, bool phase)
{
    if (precision == 4 || !variant_shape(precision, 1, variant).chunked) return 0;
    const Variant v = variant_shape(precision, 1, variant);
    const void *fn = nullptr;
    if (precision == 0) fn = th_strip_fn<double, 128, 2>(rk, phase);
    else if (v.nt == 256) fn = th_strip_fn<float, 256, 2>(rk, phase);
    else fn = th_strip_fn<float, 128, 2>(rk, phase);
    int b = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, v.nt, 0) != hipSuccess) return 0;
    return b;
}

hipError_t launch_diag(int precision, const RunDev *runs_dev, const DiagBlock *blocks, int n_blocks, int run0, int n_runs,
                       int pt, long long step, int readout, hipStream_t stream)
{
    if (n_blocks <= 0 || n_runs <= 0) return hipSuccess;
    if (precision == 4) {
        k_diag_partial<Dual><<<n_blocks, 256, 0, stream>>>(runs_dev, blocks, step, readout);
        k_diag_final<Dual><<<n_runs, 256, 0, stream>>>(runs_dev, run0, pt, step, readout);
    } else if (precision == 0) {
        k_diag_partial<double><<<n_blocks, 256, 0, stream>>>(runs_dev, blocks, step, readout);
        k_diag_final<double><<<n_runs, 256, 0, stream>>>(runs_dev, run0, pt, step, readout);
    } else {
        k_diag_partial<float><<<n_blocks, 256, 0, stream>>>(runs_dev, blocks, step, readout);
        k_diag_final<float><<<n_runs, 256, 0, stream>>>(runs_dev, run0, pt, step, readout);
    }
    return hipGetLastError();
}

// Device memory of the handles created without a caller workspace (lbm_create_static), for callers
// that cannot allocate: one copy of this array per device, held for the life of the process.  In host
// code its name is only a stand-in; kernels receive the device address found by static_workspace().
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

hipError_t static_workspace(void **ptr)
{
    static std::mutex mu;
    static std::map<int, void *> addr;   // per device
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p & 255) != 0) return hipErrorInvalidSymbol;
        it = addr.emplace(dev, p).first;
    }
    *ptr = it->second;
    return hipSuccess;
}

hipError_t launch_init(int precision, const RunDev *runs_dev, int run, long long nodes, hipStream_t stream)
{
    int blocks = (int)((nodes + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    switch (precision) {
    case 0: k_init<double><<<blocks, 256, 0, stream>>>(runs_dev, run); break;
    case 1: k_init<float><<<blocks, 256, 0, stream>>>(runs_dev, run); break;
    case 2: k_init<__half><<<blocks, 256, 0, stream>>>(runs_dev, run); break;
    case 3: k_init<__hip_bfloat16><<<blocks, 256, 0, stream>>>(runs_dev, run); break;
    case 4: k_init<Dual><<<blocks, 256, 0, stream>>>(runs_dev, run); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
