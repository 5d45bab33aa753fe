// Internal interface between the C-ABI host code (lbm_api.cpp) and the gfx950 kernels
// (lbm_kernels.hip).  Not installed; the public interface is include/lbm.h.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace lbm {

constexpr int kMaxProbes = 4096;
constexpr int kDiagBlocks = 1024;  // most diagnostic workgroups of a run
// parameter directions of the tangent precision: superheat dTr_wall, u_in, acentric factor, tau
constexpr int kTangents = 4;
// FP64 accumulators per run: [0] mass, [1] q_mean, [2] Nu, [3] sum of Nu, [4] count, [5] non-finite,
// [8 + k] dNu/dtheta_k, [12 + k] sum of dNu/dtheta_k
constexpr int kAcc = 16;
// probe limit of the tangent precision (its per-probe heat flux carries the tangents in LDS)
constexpr int kMaxTangentProbes = 1024;
// size of the per-device static workspace of handles created by lbm_create_static
constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;

// Per-run description read by every kernel.  Physical constants are kept in FP64 and converted
// to the compute type inside the kernels.
struct RunDev {
    int nx, ny, pitch;        // pitch: row stride in elements (multiple of 64)
    int bc_x;                 // 0 periodic, 1 inlet/outlet
    int cyl_x, cyl_y, cyl_r;  // cyl_r <= 0: no cylinder
    int rk;                   // 0, 2, 4
    int upwind_kind;
    int warmup;
    int np;                   // wall probes
    int pad0;
    double omega, sigma, G, gx, gy, rho_gref, rho_w, rho_l, rho_v;
    double T_sat, T_w, Tc, kappa, eos_a, eos_b, eos_R;
    double u_in, alpha, cv, shift;
    // phase-dependent transport (phase_props != 0): nu and alpha linear in rho between the vapour
    // (rho_v) and liquid (rho_l) values, held outside; alpha above is then the liquid value
    int phase_props;
    int outlet_kind;          // convective-outlet speed: 0 u_in, 1 local outflow velocity (extended launch)
    double nu_l, nu_v, alpha_v, inv_drho;   // inv_drho = 1 / (rho_l - rho_v)
    // derived on the host: 1/sqrt(Tc), 2/(G cs^2), phi'(T) = dphi_A/sqrt(T) + dphi_B, 1/cv
    double inv_sqrt_Tc, psi_scale, dphi_A, dphi_B, inv_cv;
    // derivatives of the parameter-dependent constants along the tangent directions (tangent
    // precision only; zero otherwise)
    double t_omega[kTangents], t_T_w[kTangents], t_u_in[kTangents], t_alpha[kTangents];
    double t_kappa[kTangents], t_dphi_A[kTangents], t_dphi_B[kTangents];
    void *f[2];               // populations, storage type, [9][ny][pitch]
    void *T[2];               // temperature, compute type, [ny][pitch]
    void *rho, *ux, *uy;      // macroscopic fields of the last streamed state, compute type
    void *hist[2];            // outlet history, compute type, [3][ny]
    const double *probes;     // [np][2] probe coordinates
    const void *qtab;         // compute type, [2R+3][2R+3][8] wall fractions of cut links (cyl_r > 0)
    double *partials;         // [kDiagBlocks] partial mass sums of the diagnostic workgroups
    double *acc;              // [kAcc]
    int nblk;                 // diagnostic workgroups of this run (<= kDiagBlocks)
    int diag_every, check_every;
};

// One workgroup of the diagnostic reduction: rows [row0, row1) of run `run`, its index among the
// run's workgroups.
struct DiagBlock {
    int run, row0, row1, index;
};

// One work item: run index and tile coordinates.
struct Tile {
    int run, tx, ty, pad;
};

// Launch variant of a stencil kernel: tile of tx x ty nodes per workgroup of nt threads.
struct Variant {
    int tx, ty, nt;
    int min_waves;  // > 0: compiled with a register budget for this many waves per SIMD
    // 1: a strip of tx columns marching down a chunk of rows; its tile entry carries the chunk's
    // first row (ty) and row count (pad, a multiple of 8): ty rows, or with ty = 0 as many as spread
    // the strips of a launch over the workgroups the GPU holds at once
    int chunked;
};

// kernel: 0 = stream+collide (k_lbm), 1 = temperature update (k_thermal)
int variant_count(int precision, int kernel);
// workgroups of a chunked temperature variant that one CU holds at once (0 if not chunked)
int chunked_blocks_per_cu(int precision, int variant, int rk, bool phase);
Variant variant_shape(int precision, int kernel, int v);

// Start / stop events filled in by a kernel's own dispatch (timing inside the step sequence).
struct Timing {
    hipEvent_t start, stop;
};

// Device address of the current device's static workspace (kStaticWorkspaceBytes, 256-byte
// aligned), looked up once per device.
hipError_t static_workspace(void **ptr);

// Launchers (each enqueues on `stream`; returns a hipError_t).
hipError_t launch_init(int precision, const RunDev *runs_dev, int run, long long nodes, hipStream_t stream);
// phase: some run of the launch has phase-dependent transport or a heated wall (FP32 / FP64
// only); the kernels without these features are launched otherwise.  timing (optional): events
// that take the start and end timestamps of this dispatch.
hipError_t launch_lbm(int precision, int variant, bool write_f, bool phase, const RunDev *runs_dev, const Tile *tiles,
                      int n_tiles, int parity_f, int parity_t, int parity_h, long long step, hipStream_t stream,
                      const Timing *timing = nullptr);
hipError_t launch_thermal(int precision, int rk, int variant, bool phase, const RunDev *runs_dev, const Tile *tiles,
                          int n_tiles, int parity_t, long long step, hipStream_t stream, const Timing *timing = nullptr);
// Diagnostic reduction (two launches) of runs run0 .. run0 + n_runs - 1 over their workgroups
// blocks[0 .. n_blocks): with readout < 0 the runs whose Nu sample or finiteness check falls on
// `step` (accumulating the Nu samples), else a read-out of run `readout`.
hipError_t launch_diag(int precision, const RunDev *runs_dev, const DiagBlock *blocks, int n_blocks, int run0, int n_runs,
                       int parity_t, long long step, int readout, hipStream_t stream);

// Reverse-mode adjoint of one FP64 step of run `run` (lbm_adjoint.hip).  Rh: host copy of the run's
// descriptor.  fs, hist, T: state n; ain / aout: adjoint states of n+1 / n (adjoint_state_doubles);
// scratch: adjoint_scratch_doubles doubles.
size_t adjoint_scratch_doubles(int nx, int ny, int pitch);
size_t adjoint_state_doubles(int nx, int ny, int pitch);
hipError_t launch_adjoint_step(const RunDev *runs_dev, int run, const RunDev &Rh, const double *fs, const double *hist,
                               const double *T, const double *ain, double *aout, double *scratch, long long step,
                               double nu_weight, hipStream_t stream);
// adds the initial state's parameter dependence to the accumulated gradient of the adjoint state adj
hipError_t launch_adjoint_initial(const RunDev *runs_dev, int run, double *adj, bool default_state, hipStream_t stream);

}  // namespace lbm
