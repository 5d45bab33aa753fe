// Host side of the C ABI declared in include/lbm.h: configuration checks, derived constants,
// workspace carving, launch sequencing and host read-back.  All device work is enqueued on the
// caller's stream; the library never allocates device memory.
#include "lbm.h"
#include "lbm_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

using lbm::RunDev;
using lbm::Tile;

// A captured window of steps, replayed while the launch pattern repeats.
struct StepGraph {
    int pf, pt, ph, length;
    int groups;  // stream groups the window was captured with (0: one stream)
    long long phase;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

struct lbm_handle {
    int n_runs = 0;
    int precision = 0;
    int rk = 0;
    hipStream_t stream = nullptr;
    std::vector<lbm_config> cfgs;
    std::vector<RunDev> runs;         // host copies of the device descriptors
    RunDev *runs_dev = nullptr;
    Tile *tiles_lbm = nullptr, *tiles_th = nullptr;
    int cap_lbm = 0, cap_th = 0;      // tile-table capacities (largest over the variants)
    std::vector<int> lbm_off, lbm_cnt, th_off, th_cnt;
    int n_lbm = 0, n_th = 0;
    lbm::DiagBlock *diag_blocks = nullptr;  // diagnostic workgroups, run by run
    std::vector<int> diag_off, diag_cnt;
    int var[2] = {0, 0};              // launch variant of k_lbm, k_thermal
    bool phase = false;               // some run has phase-dependent transport or a heated wall
    int pf = 0, pt = 0, ph = 0;
    long long step = 0;
    bool use_graphs = true;
    bool tune_steps = false;  // LBM_OPT_TUNE_STEPS: lbm_autotune times whole steps
    std::vector<StepGraph> graphs;
    // per run: still in the default state of lbm_create (its initial fields depend on u_in)
    std::vector<char> default_state;
    // stream groups (LBM_OPT_STREAM_GROUPS > 1): contiguous ranges of runs stepped on streams of their
    // own, so that one group's temperature update overlaps another group's streaming
    struct Group {
        int run0, run1;          // runs [run0, run1)
        hipStream_t s;
        hipEvent_t done;
    };
    std::vector<Group> groups;
    hipEvent_t fork = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream used only to record graphs
    // lbm_create_static: the workspace is the device's static array, valid until the next
    // lbm_create_static on that device (generation `gen`)
    bool static_ws = false;
    int device = -1;  // the device current at creation
    unsigned long long gen = 0;
    std::string err;
};

namespace {

std::string g_create_error;

// Optional roctx ranges around the host entry points (seen by rocprofv3 --marker-trace): the ROCm
// roctx library is loaded at run time if present; without it the ranges are no-ops.
struct Roctx {
    int (*push)(const char *) = nullptr;
    int (*pop)() = nullptr;
    Roctx()
    {
        for (const char *name : {"librocprofiler-sdk-roctx.so.1", "libroctx64.so.4"}) {
            void *lib = dlopen(name, RTLD_NOW | RTLD_LOCAL);
            if (!lib) continue;
            push = (int (*)(const char *))dlsym(lib, "roctxRangePushA");
            pop = (int (*)())dlsym(lib, "roctxRangePop");
            if (push && pop) return;
            push = nullptr;
            pop = nullptr;
        }
    }
};

struct Range {
    const Roctx &r;
    explicit Range(const char *name) : r(roctx())
    {
        if (r.push) r.push(name);
    }
    ~Range()
    {
        if (r.pop) r.pop();
    }
    static const Roctx &roctx()
    {
        static const Roctx instance;
        return instance;
    }
};

int fail(lbm_handle *h, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    else g_create_error = buf;
    return code;
}

#define HIPCHK(h, call)                                                                       \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(h, LBM_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
int pitch_of(int nx) { return (nx + 63) / 64 * 64; }
// bytes per stored population / per compute-type value; the tangent precision stores an FP64
// value followed by its kTangents derivatives
constexpr size_t kDualBytes = 8 * (1 + lbm::kTangents);
size_t storage_bytes(int precision)
{
    return precision == 4 ? kDualBytes : (precision == 0 ? 8 : (precision == 1 ? 4 : 2));
}
size_t compute_bytes(int precision) { return precision == 4 ? kDualBytes : (precision == 0 ? 8 : 4); }
int probe_count(int r) { return r > 0 ? 8 * (int)std::ceil(M_PI * r / 4.0) : 0; }

// ---- Peng-Robinson thermodynamics on the host (set-up only) -----------------------------------
struct PR {
    double a, b, R, kappa, Tc;
    explicit PR(const lbm_config &c)
        : a(c.eos_a), b(c.eos_b), R(c.eos_R),
          kappa(0.37464 + 1.54226 * c.acentric - 0.26992 * c.acentric * c.acentric),
          Tc(0.0778 * c.eos_a / (0.4572 * c.eos_b * c.eos_R)) {}
    double phi(double T) const { double s = 1.0 + kappa * (1.0 - std::sqrt(T / Tc)); return s * s; }
    // pressure as a function of specific volume v = 1/rho
    double p_v(double v, double T) const { return R * T / (v - b) - a * phi(T) / (v * v + 2.0 * b * v - b * b); }
    double dp_dv(double v, double T) const
    {
        double d = v * v + 2.0 * b * v - b * b;
        return -R * T / ((v - b) * (v - b)) + a * phi(T) * (2.0 * v + 2.0 * b) / (d * d);
    }
    // integral of p dv
    double P_int(double v, double T) const
    {
        double s2 = std::sqrt(2.0);
        return R * T * std::log(v - b) - a * phi(T) / (2.0 * s2 * b) * std::log((v + b - s2 * b) / (v + b + s2 * b));
    }
};

// Maxwell construction: equal area under the isotherm p(v) between the liquid and vapour
// volumes.  The two spinodal volumes bracket the loop; for a trial pressure the outer roots are
// found by bisection on the monotone branches and the pressure is adjusted by bisection until
// the area between the isotherm and the horizontal line vanishes.
bool maxwell(const PR &pr, double T, double &rho_v, double &rho_l)
{
    const double vmin = pr.b * 1.000001, vmax = 1e6;
    // spinodals: sign changes of dp/dv on a logarithmic scan of v
    std::vector<double> sp;
    const int N = 40000;
    double lv0 = std::log(vmin), lv1 = std::log(vmax);
    double prev_v = vmin, prev_d = pr.dp_dv(vmin, T);
    for (int k = 1; k <= N && sp.size() < 2; ++k) {
        double v = std::exp(lv0 + (lv1 - lv0) * k / N);
        double d = pr.dp_dv(v, T);
        if ((d > 0) != (prev_d > 0)) {
            double lo = prev_v, hi = v, dlo = prev_d;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi), dm = pr.dp_dv(mid, T);
                if ((dm > 0) == (dlo > 0)) { lo = mid; dlo = dm; } else hi = mid;
            }
            sp.push_back(0.5 * (lo + hi));
        }
        prev_v = v;
        prev_d = d;
    }
    if (sp.size() < 2) return false;
    const double v_sl = sp[0], v_sv = sp[1];  // liquid spinodal (smaller v), vapour spinodal
    double plo = std::max(pr.p_v(v_sl, T), 1e-14), phi_ = pr.p_v(v_sv, T);
    auto root = [&](double p, double lo, double hi) {
        double flo = pr.p_v(lo, T) - p;
        for (int it = 0; it < 300; ++it) {
            double mid = 0.5 * (lo + hi), fm = pr.p_v(mid, T) - p;
            if ((fm > 0) == (flo > 0)) { lo = mid; flo = fm; } else hi = mid;
        }
        return 0.5 * (lo + hi);
    };
    double vl = 0, vv = 0;
    for (int it = 0; it < 200; ++it) {
        double p = 0.5 * (plo + phi_);
        vl = root(p, vmin, v_sl);
        vv = root(p, v_sv, vmax);
        double area = pr.P_int(vv, T) - pr.P_int(vl, T) - p * (vv - vl);
        if (area > 0) plo = p; else phi_ = p;
    }
    rho_l = 1.0 / vl;
    rho_v = 1.0 / vv;
    return true;
}

int validate(const lbm_config *c, int n, int *prec, int *rk, lbm_handle *h)
{
    if (!c || n <= 0) return fail(h, LBM_EINVAL, "no run configurations");
    for (int r = 0; r < n; ++r) {
        const lbm_config &k = c[r];
        if (k.nx < 4 || k.ny < 4) return fail(h, LBM_EINVAL, "run %d: grid must be at least 4x4", r);
        if (9.0 * k.ny * pitch_of(k.nx) * storage_bytes(k.precision) >= 4294967296.0)
            return fail(h, LBM_EINVAL, "run %d: grid too large (9 population planes must stay below 4 GiB)", r);
        if (k.bc_x != LBM_BC_PERIODIC && k.bc_x != LBM_BC_INLET_OUTLET && k.bc_x != LBM_BC_WALL_OUTLET)
            return fail(h, LBM_EINVAL, "run %d: bad bc_x", r);
        if (k.precision < 0 || k.precision > 4) return fail(h, LBM_EINVAL, "run %d: bad precision", r);
        if (k.outlet_kind != LBM_OUTLET_U_IN && k.outlet_kind != LBM_OUTLET_LOCAL)
            return fail(h, LBM_EINVAL, "run %d: bad outlet_kind", r);
        if (k.precision >= 2 && (k.nu_vapor > 0 || k.alpha_vapor > 0 || k.bc_x == LBM_BC_WALL_OUTLET ||
                                 k.outlet_kind != LBM_OUTLET_U_IN))
            return fail(h, LBM_EINVAL,
                        "run %d: phase-dependent transport, the heated wall and the local outlet speed need FP64 or FP32", r);
        if (k.precision == 4 && probe_count(k.cyl_r) > lbm::kMaxTangentProbes)
            return fail(h, LBM_EINVAL, "run %d: cylinder too large for the tangent precision", r);
        if (k.precision != c[0].precision) return fail(h, LBM_EINVAL, "all runs must share one precision");
        if (k.rk_stages != 0 && k.rk_stages != 2 && k.rk_stages != 4) return fail(h, LBM_EINVAL, "run %d: rk_stages must be 0, 2 or 4", r);
        if (k.rk_stages != c[0].rk_stages) return fail(h, LBM_EINVAL, "all runs must share rk_stages");
        if (!(k.nu > 0)) return fail(h, LBM_EINVAL, "run %d: nu must be positive", r);
        if (k.G == 0) return fail(h, LBM_EINVAL, "run %d: G must be nonzero", r);
        if (k.rk_stages > 0 && !(k.cv > 0 && k.alpha_T >= 0)) return fail(h, LBM_EINVAL, "run %d: bad thermal constants", r);
        if (!(k.eos_a > 0 && k.eos_b > 0 && k.eos_R > 0 && k.Tr_sat > 0)) return fail(h, LBM_EINVAL, "run %d: bad EOS constants", r);
        if (k.warmup_steps < 0 || k.diag_every < 0 || k.check_every < 0) return fail(h, LBM_EINVAL, "run %d: negative counter", r);
        if (k.cyl_r > 0) {
            if (k.cyl_x - k.cyl_r < 3 || k.cyl_x + k.cyl_r > k.nx - 4 || k.cyl_y - k.cyl_r < 2 || k.cyl_y + k.cyl_r > k.ny - 3)
                return fail(h, LBM_EINVAL, "run %d: cylinder too close to the domain edge", r);
            if (probe_count(k.cyl_r) > lbm::kMaxProbes) return fail(h, LBM_EINVAL, "run %d: cylinder too large", r);
        }
    }
    *prec = c[0].precision;
    *rk = c[0].rk_stages;
    return LBM_OK;
}

// rows per diagnostic workgroup of a run: at most kDiagBlocks workgroups, at least ~2048 nodes each
int diag_rows(const lbm_config &k)
{
    const int a = (k.ny + lbm::kDiagBlocks - 1) / lbm::kDiagBlocks, b = (2048 + k.nx - 1) / k.nx;
    return std::max(1, std::max(a, b));
}
int diag_count(const lbm_config &k) { return (k.ny + diag_rows(k) - 1) / diag_rows(k); }

struct Layout {
    size_t runs_off, tiles_lbm_off, tiles_th_off, diag_off, total;
    std::vector<size_t> run_off;
    int n_lbm, n_th;
};

// entries of the cut-link table: 8 directions per node of the box |x - x_c|, |y - y_c| <= R + 1
size_t qtab_count(int cyl_r) { return cyl_r > 0 ? (size_t)(2 * cyl_r + 3) * (2 * cyl_r + 3) * 8 : 0; }

size_t run_bytes(const lbm_config &k)
{
    const size_t plane = (size_t)k.ny * pitch_of(k.nx);
    const size_t sb = storage_bytes(k.precision), cb = compute_bytes(k.precision);
    size_t b = 0;
    b += 2 * align256(9 * plane * sb);                      // f[2]
    b += 5 * align256(plane * cb);                          // T[2], rho, ux, uy
    b += 2 * align256(3 * (size_t)k.ny * cb);               // hist[2]
    b += align256(2 * sizeof(double) * std::max(1, probe_count(k.cyl_r)));  // probes
    b += align256(sizeof(double) * lbm::kDiagBlocks);       // partials
    b += align256(sizeof(double) * lbm::kAcc);              // acc
    b += align256(qtab_count(k.cyl_r) * cb);                // wall fractions of cut links
    return b;
}

// rows of the chunks of a chunked variant: ty rounded up to a whole number of ring periods (8 rows),
// or for ty = 0 the run's rows split into n_chunks
int chunk_rows(const lbm::Variant &v, int ny, int n_chunks)
{
    const int ch = v.ty > 0 ? v.ty : (ny + n_chunks - 1) / n_chunks;
    return std::max(8, (ch + 7) / 8 * 8);
}

// tiles of a variant over the runs (for a chunked variant whose chunks are sized at build time, the
// most there can be: chunks of 8 rows)
int tile_count(const lbm_config *c, int n, lbm::Variant v)
{
    int t = 0;
    for (int r = 0; r < n; ++r) {
        const int ty = v.chunked ? chunk_rows(v, c[r].ny, (c[r].ny + 7) / 8) : v.ty;
        t += ((c[r].nx + v.tx - 1) / v.tx) * ((c[r].ny + ty - 1) / ty);
    }
    return t;
}

Layout layout(const lbm_config *c, int n)
{
    Layout L;
    L.n_lbm = L.n_th = 0;
    for (int k = 0; k < 2; ++k)
        for (int v = 0; v < lbm::variant_count(c[0].precision, k); ++v) {
            const int t = tile_count(c, n, lbm::variant_shape(c[0].precision, k, v));
            if (k == 0) L.n_lbm = std::max(L.n_lbm, t);
            else L.n_th = std::max(L.n_th, t);
        }
    size_t off = 0;
    L.runs_off = off; off += align256(sizeof(RunDev) * n);
    L.tiles_lbm_off = off; off += align256(sizeof(Tile) * L.n_lbm);
    L.tiles_th_off = off; off += align256(sizeof(Tile) * L.n_th);
    int nd = 0;
    for (int r = 0; r < n; ++r) nd += diag_count(c[r]);
    L.diag_off = off; off += align256(sizeof(lbm::DiagBlock) * nd);
    for (int r = 0; r < n; ++r) { L.run_off.push_back(off); off += run_bytes(c[r]); }
    L.total = off;
    return L;
}

double ld_storage(const unsigned char *p, int prec, size_t k)
{
    switch (prec) {
    case 4: return ((const double *)p)[k * (1 + lbm::kTangents)];
    case 0: return ((const double *)p)[k];
    case 1: return ((const float *)p)[k];
    case 2: return (double)__half2float(((const __half *)p)[k]);
    default: return (double)__bfloat162float(((const __hip_bfloat16 *)p)[k]);
    }
}

void st_storage(unsigned char *p, int prec, size_t k, double v)
{
    switch (prec) {
    case 4:
        ((double *)p)[k * (1 + lbm::kTangents)] = v;
        for (int d = 1; d <= lbm::kTangents; ++d) ((double *)p)[k * (1 + lbm::kTangents) + d] = 0.0;
        break;
    case 0: ((double *)p)[k] = v; break;
    case 1: ((float *)p)[k] = (float)v; break;
    case 2: ((__half *)p)[k] = __float2half_rn((float)v); break;
    default: ((__hip_bfloat16 *)p)[k] = __float2bfloat16((float)v); break;
    }
}

double ld_compute(const unsigned char *p, int prec, size_t k)
{
    if (prec == 4) return ((const double *)p)[k * (1 + lbm::kTangents)];
    return prec == 0 ? ((const double *)p)[k] : (double)((const float *)p)[k];
}

// store v (tangent precision: with zero derivatives, or derivative 1 along direction seed_dir)
void st_compute(unsigned char *p, int prec, size_t k, double v, int seed_dir = -1)
{
    if (prec == 4) {
        double *e = (double *)p + k * (1 + lbm::kTangents);
        e[0] = v;
        for (int d = 0; d < lbm::kTangents; ++d) e[1 + d] = d == seed_dir ? 1.0 : 0.0;
    } else if (prec == 0) {
        ((double *)p)[k] = v;
    } else {
        ((float *)p)[k] = (float)v;
    }
}

const double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

bool solid_host(const RunDev &R, int x, int y)
{
    if (R.cyl_r <= 0) return false;
    long dx = x - R.cyl_x, dy = y - R.cyl_y;
    return dx * dx + dy * dy <= (long)R.cyl_r * R.cyl_r;
}

// Wall fraction of the link from fluid node (x, y) along -c_i into the cylinder: the smaller root
// q of |d - q c_i|^2 = R^2 with d the node's offset from the centre (linear interpolated
// bounce-back, Sec. IV A).  Tabulated in the compute type with its branch folded in (see fix_near
// in the kernels): 0 = plain pull, 2q in (0,1) or 4 for q < 1/2 (with / without a fluid node at
// x + c_i), -2q for q >= 1/2.
std::vector<unsigned char> cut_link_table(const RunDev &R, int prec)
{
    const size_t n = qtab_count(R.cyl_r);
    std::vector<unsigned char> out(n * compute_bytes(prec), 0);
    if (!n) return out;
    static const int cx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1}, cy[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    const int bw = 2 * R.cyl_r + 3, bx0 = R.cyl_x - R.cyl_r - 1, by0 = R.cyl_y - R.cyl_r - 1;
    for (int by = 0; by < bw; ++by)
        for (int bx = 0; bx < bw; ++bx) {
            const int x = bx0 + bx, y = by0 + by;
            if (solid_host(R, x, y)) continue;
            for (int i = 1; i < 9; ++i) {
                if (!solid_host(R, x - cx[i], y - cy[i])) continue;
                const double dx = x - R.cyl_x, dy = y - R.cyl_y;
                const double c2 = cx[i] * cx[i] + cy[i] * cy[i], dc = dx * cx[i] + dy * cy[i];
                const double Rr = R.cyl_r;
                const double disc = dc * dc - c2 * (dx * dx + dy * dy - Rr * Rr);
                const double q = (dc - std::sqrt(disc)) / c2;
                double v;
                if (q < 0.5) v = solid_host(R, x + cx[i], y + cy[i]) ? 4.0 : 2.0 * q;
                else v = -(2.0 * q);
                st_compute(out.data(), prec, (size_t)(by * bw + bx) * 8 + (i - 1), v);
            }
        }
    return out;
}

// XCD-aware order of one run's tiles (row-major on entry): block b runs on XCD b mod 8, so each XCD
// receives a contiguous band of tiles (their shared halos stay in one L2).  Within a band the tiles
// for which first(tile) holds are dispatched first: the stream-and-collide tiles next to the cylinder,
// which take a second memory round trip, then start in the first wave of workgroups instead of
// finishing last.
template <typename First>
void xcd_order(std::vector<Tile> &tiles, size_t off, size_t n, First first)
{
    const size_t nx = 8;
    if (n < 2 * nx || n % nx != 0) return;
    std::vector<Tile> band(tiles.begin() + off, tiles.begin() + off + n);
    const size_t chunk = n / nx;
    for (size_t j = 0; j < nx; ++j)
        std::stable_partition(band.begin() + j * chunk, band.begin() + (j + 1) * chunk, first);
    for (size_t t = 0; t < n; ++t) {
        const size_t j = t / chunk, k = t % chunk;
        tiles[off + k * nx + j] = band[t];
    }
}

int max_warmup(const lbm_handle *h)
{
    int m = 0;
    for (const auto &k : h->cfgs) m = std::max(m, k.warmup_steps);
    return m;
}

void drop_graphs(lbm_handle *h)
{
    for (auto &g : h->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    h->graphs.clear();
}

// Build and upload the tile tables of the current launch variants (per-run contiguous ranges,
// XCD-grouped order inside each range).
int build_tiles(lbm_handle *h)
{
    std::vector<Tile> tl[2];
    for (int k = 0; k < 2; ++k) {
        const lbm::Variant v = lbm::variant_shape(h->precision, k, h->var[k]);
        std::vector<int> &off = k == 0 ? h->lbm_off : h->th_off;
        std::vector<int> &cnt = k == 0 ? h->lbm_cnt : h->th_cnt;
        off.clear();
        cnt.clear();
        // chunks sized to the launch: the workgroups the GPU holds at once, shared among the runs in
        // proportion to their nodes, each run's strips taking an equal number of chunks
        double resident = 0.0, nodes = 0.0;
        if (v.chunked && v.ty == 0) {
            int cus = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) cus = 0;
            resident = (double)cus * lbm::chunked_blocks_per_cu(h->precision, h->var[k], h->rk, h->phase);
            for (int r = 0; r < h->n_runs; ++r) nodes += (double)h->runs[r].nx * h->runs[r].ny;
        }
        for (int r = 0; r < h->n_runs; ++r) {
            const RunDev &R = h->runs[r];
            off.push_back((int)tl[k].size());
            const int strips = (R.nx + v.tx - 1) / v.tx;
            if (v.chunked) {
                const double share = resident * ((double)R.nx * R.ny / std::max(nodes, 1.0)) / strips;
                const int ch = chunk_rows(v, R.ny, std::max(1, std::min((R.ny + 7) / 8, (int)share)));
                for (int y0 = 0; y0 < R.ny; y0 += ch)
                    for (int tx = 0; tx < strips; ++tx) tl[k].push_back(Tile{r, tx, y0, ch});
            } else {
                for (int ty = 0; ty < (R.ny + v.ty - 1) / v.ty; ++ty)
                    for (int tx = 0; tx < strips; ++tx) tl[k].push_back(Tile{r, tx, ty, 0});
            }
            cnt.push_back((int)tl[k].size() - off.back());
            // stream-and-collide tiles whose region (tile + the 2-node psi halo) meets the cut-link box or
            // the outlet column (whose convective condition reads the outlet history after the pulls)
            const int bx0 = R.cyl_x - R.cyl_r - 1, bx1 = R.cyl_x + R.cyl_r + 1;
            const int by0 = R.cyl_y - R.cyl_r - 1, by1 = R.cyl_y + R.cyl_r + 1;
            auto near = [&](const Tile &t) {
                if (k != 0) return false;
                const int x0 = t.tx * v.tx - 2, x1 = (t.tx + 1) * v.tx + 1, y0 = t.ty * v.ty - 2, y1 = (t.ty + 1) * v.ty + 1;
                if (R.bc_x != 0 && x1 >= R.nx - 1) return true;
                return R.cyl_r > 0 && x1 >= bx0 && x0 <= bx1 && y1 >= by0 && y0 <= by1;
            };
            xcd_order(tl[k], off.back(), cnt.back(), near);
        }
    }
    if ((int)tl[0].size() > h->cap_lbm || (int)tl[1].size() > h->cap_th) return fail(h, LBM_EINVAL, "tile table overflow");
    h->n_lbm = (int)tl[0].size();
    h->n_th = (int)tl[1].size();
    HIPCHK(h, hipMemcpyAsync(h->tiles_lbm, tl[0].data(), sizeof(Tile) * tl[0].size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->tiles_th, tl[1].data(), sizeof(Tile) * tl[1].size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    drop_graphs(h);
    return LBM_OK;
}

// generation of each device's static workspace: bumped by every lbm_create_static on the device
std::mutex g_static_mu;
std::map<int, unsigned long long> g_static_gen;

// a NULL handle is invalid; a static-workspace handle whose memory a later lbm_create_static on its
// device took over may no longer launch anything
int check_handle(lbm_handle *h)
{
    if (!h) return LBM_EINVAL;
    if (h->static_ws) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (g_static_gen[h->device] != h->gen)
            return fail(h, LBM_ESTATE, "the static workspace of device %d now belongs to a later lbm_create_static",
                        h->device);
    }
    return LBM_OK;
}

int check_run(lbm_handle *h, int run)
{
    if (int rc = check_handle(h)) return rc;
    if (run < 0 || run >= h->n_runs) return fail(h, LBM_EINVAL, "run index %d out of range", run);
    return LBM_OK;
}

// upload host fields (double, [ny][nx]) into a pitched compute-type plane; seed_dir >= 0 gives
// the values derivative 1 along that tangent direction
int upload_plane(lbm_handle *h, const RunDev &R, void *dst, const double *src, double fill, int seed_dir = -1)
{
    const size_t cb = compute_bytes(h->precision);
    std::vector<unsigned char> buf((size_t)R.ny * R.pitch * cb, 0);
    for (int y = 0; y < R.ny; ++y)
        for (int x = 0; x < R.nx; ++x)
            st_compute(buf.data(), h->precision, (size_t)y * R.pitch + x, src ? src[(size_t)y * R.nx + x] : fill,
                       seed_dir);
    HIPCHK(h, hipMemcpyAsync(dst, buf.data(), buf.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int download_plane(lbm_handle *h, const RunDev &R, const void *src, std::vector<double> &out)
{
    const size_t cb = compute_bytes(h->precision);
    std::vector<unsigned char> buf((size_t)R.ny * R.pitch * cb);
    HIPCHK(h, hipMemcpyAsync(buf.data(), src, buf.size(), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    out.resize((size_t)R.nx * R.ny);
    for (int y = 0; y < R.ny; ++y)
        for (int x = 0; x < R.nx; ++x) out[(size_t)y * R.nx + x] = ld_compute(buf.data(), h->precision, (size_t)y * R.pitch + x);
    return LBM_OK;
}

// macroscopic pass of one run without collision (writes rho, ux, uy of the current state)
int moments_pass(lbm_handle *h, int run)
{
    HIPCHK(h, lbm::launch_lbm(h->precision, h->var[0], false, h->phase, h->runs_dev, h->tiles_lbm + h->lbm_off[run],
                              h->lbm_cnt[run], h->pf, h->pt, h->ph, h->step, h->stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_config *cfgs, int n_runs)
{
    int prec, rk;
    if (validate(cfgs, n_runs, &prec, &rk, nullptr) != LBM_OK) return 0;
    return layout(cfgs, n_runs).total;
}

static int set_fields_impl(lbm_handle *h, int run, const double *rho, const double *ux, const double *uy,
                           const double *T, int ux_seed_dir);

static int create_impl(const lbm_config *cfgs, int n_runs, void *dev_workspace, size_t ws_bytes, void *hip_stream,
                       lbm_handle **out, int static_device);

int lbm_create(const lbm_config *cfgs, int n_runs, void *dev_workspace, size_t ws_bytes, void *hip_stream,
               lbm_handle **out)
{
    return create_impl(cfgs, n_runs, dev_workspace, ws_bytes, hip_stream, out, -1);
}

int lbm_create_static(const lbm_config *cfgs, int n_runs, void *hip_stream, lbm_handle **out)
{
    const Range range("lbm_create_static");
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int prec, rk;
    int rc = validate(cfgs, n_runs, &prec, &rk, nullptr);
    if (rc != LBM_OK) return rc;
    const size_t need = layout(cfgs, n_runs).total;
    if (need > lbm::kStaticWorkspaceBytes)
        return fail(nullptr, LBM_ENOMEM, "the runs need %zu bytes of workspace, more than the %zu of the static workspace",
                    need, lbm::kStaticWorkspaceBytes);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, LBM_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    void *ws = nullptr;
    e = lbm::static_workspace(&ws);
    if (e != hipSuccess) return fail(nullptr, LBM_EDEVICE, "static workspace: %s", hipGetErrorString(e));
    // the array is shared by every static handle of this device: earlier ones stop here
    (void)hipDeviceSynchronize();
    return create_impl(cfgs, n_runs, ws, lbm::kStaticWorkspaceBytes, hip_stream, out, dev);
}

static int create_impl(const lbm_config *cfgs, int n_runs, void *dev_workspace, size_t ws_bytes, void *hip_stream,
                       lbm_handle **out, int static_device)
{
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int prec, rk;
    int rc = validate(cfgs, n_runs, &prec, &rk, nullptr);
    if (rc != LBM_OK) return rc;
    const Layout L = layout(cfgs, n_runs);
    if (!dev_workspace || ws_bytes < L.total) return fail(nullptr, LBM_ENOMEM, "workspace needs %zu bytes", L.total);
    if (((uintptr_t)dev_workspace & 255) != 0) return fail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");

    lbm_handle *h = new lbm_handle();
    if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
    if (static_device >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        h->static_ws = true;
        h->device = static_device;
        h->gen = ++g_static_gen[static_device];
    }
    h->n_runs = n_runs;
    h->precision = prec;
    h->rk = rk;
    h->stream = (hipStream_t)hip_stream;
    h->cfgs.assign(cfgs, cfgs + n_runs);
    unsigned char *ws = (unsigned char *)dev_workspace;
    h->runs_dev = (RunDev *)(ws + L.runs_off);
    h->tiles_lbm = (Tile *)(ws + L.tiles_lbm_off);
    h->tiles_th = (Tile *)(ws + L.tiles_th_off);
    h->diag_blocks = (lbm::DiagBlock *)(ws + L.diag_off);
    h->cap_lbm = L.n_lbm;
    h->cap_th = L.n_th;
    std::vector<std::vector<double>> probes(n_runs);

    for (int r = 0; r < n_runs; ++r) {
        const lbm_config &k = cfgs[r];
        RunDev R;
        std::memset(&R, 0, sizeof(R));
        R.nx = k.nx; R.ny = k.ny; R.pitch = pitch_of(k.nx); R.bc_x = k.bc_x;
        R.cyl_x = k.cyl_x; R.cyl_y = k.cyl_y; R.cyl_r = k.cyl_r;
        R.rk = k.rk_stages; R.upwind_kind = k.upwind_kind; R.warmup = k.warmup_steps;
        R.np = probe_count(k.cyl_r);
        PR pr(k);
        R.Tc = pr.Tc;
        R.kappa = pr.kappa;
        R.T_sat = k.Tr_sat * pr.Tc;
        R.T_w = R.T_sat + k.dTr_wall * pr.Tc;
        double rl = k.rho_l, rv = k.rho_v;
        if (rl <= 0 || rv <= 0) {
            if (!maxwell(pr, R.T_sat, rv, rl)) {
                delete h;
                return fail(nullptr, LBM_EINVAL, "run %d: no liquid-vapour coexistence at T_sat", r);
            }
        }
        R.rho_l = rl; R.rho_v = rv;
        R.inv_drho = 1.0 / (rl - rv);
        R.rho_w = k.rho_wall > 0 ? k.rho_wall : rl;
        R.rho_gref = k.rho_gref >= 0 ? k.rho_gref : rl;
        R.omega = 1.0 / (k.nu / (1.0 / 3.0) + 0.5);
        R.sigma = k.sigma; R.G = k.G; R.gx = k.gx; R.gy = k.gy;
        R.eos_a = k.eos_a; R.eos_b = k.eos_b; R.eos_R = k.eos_R;
        R.u_in = k.u_in; R.alpha = k.alpha_T; R.cv = k.cv;
        R.phase_props = (k.nu_vapor > 0 || k.alpha_vapor > 0) ? 1 : 0;
        R.outlet_kind = k.outlet_kind;
        h->phase |= R.phase_props != 0 || R.bc_x == LBM_BC_WALL_OUTLET || R.outlet_kind != LBM_OUTLET_U_IN;
        R.nu_l = k.nu;
        R.nu_v = k.nu_vapor > 0 ? k.nu_vapor : k.nu;
        R.alpha_v = k.alpha_vapor > 0 ? k.alpha_vapor : k.alpha_T;
        R.shift = prec >= 2 ? (k.rho_ref_shift > 0 ? k.rho_ref_shift : rl) : 0.0;
        R.inv_sqrt_Tc = 1.0 / std::sqrt(R.Tc);
        R.psi_scale = 2.0 / (R.G * (1.0 / 3.0));
        R.dphi_A = -R.kappa * (1.0 + R.kappa) / std::sqrt(R.Tc);
        R.dphi_B = R.kappa * R.kappa / R.Tc;
        R.inv_cv = 1.0 / R.cv;
        {
            // derivatives of the parameter-dependent constants (read by the tangent precision and by
            // the adjoint of FP64 runs) along the directions: 0 superheat dTr_wall, 1 u_in, 2 acentric
            // factor, 3 tau (at fixed nu/alpha ratio); the coexistence densities, T_sat and the other
            // constants are held
            const double tau = k.nu / (1.0 / 3.0) + 0.5;
            const double dkappa = 1.54226 - 2.0 * 0.26992 * k.acentric;
            R.t_T_w[0] = pr.Tc;
            R.t_u_in[1] = 1.0;
            R.t_kappa[2] = dkappa;
            R.t_dphi_A[2] = -(1.0 + 2.0 * R.kappa) / std::sqrt(R.Tc) * dkappa;
            R.t_dphi_B[2] = 2.0 * R.kappa / R.Tc * dkappa;
            R.t_omega[3] = -1.0 / (tau * tau);
            R.t_alpha[3] = R.alpha / (tau - 0.5);
        }

        unsigned char *p = ws + L.run_off[r];
        const size_t plane = (size_t)R.ny * R.pitch;
        const size_t sb = storage_bytes(prec), cb = compute_bytes(prec);
        for (int b = 0; b < 2; ++b) { R.f[b] = p; p += align256(9 * plane * sb); }
        for (int b = 0; b < 2; ++b) { R.T[b] = p; p += align256(plane * cb); }
        R.rho = p; p += align256(plane * cb);
        R.ux = p; p += align256(plane * cb);
        R.uy = p; p += align256(plane * cb);
        for (int b = 0; b < 2; ++b) { R.hist[b] = p; p += align256(3 * (size_t)R.ny * cb); }
        R.probes = (const double *)p; p += align256(2 * sizeof(double) * std::max(1, R.np));
        R.partials = (double *)p; p += align256(sizeof(double) * lbm::kDiagBlocks);
        R.acc = (double *)p; p += align256(sizeof(double) * lbm::kAcc);
        R.nblk = diag_count(k);
        R.diag_every = k.diag_every;
        R.check_every = k.check_every;
        R.qtab = qtab_count(R.cyl_r) ? p : nullptr; p += align256(qtab_count(R.cyl_r) * cb);
        h->runs.push_back(R);

        // probe ring at radius R + 1.5
        probes[r].resize(2 * std::max(1, R.np));
        for (int q = 0; q < R.np; ++q) {
            double th = 2.0 * M_PI * (q + 0.5) / R.np, rr = R.cyl_r + 1.5;
            probes[r][2 * q] = R.cyl_x + rr * std::cos(th);
            probes[r][2 * q + 1] = R.cyl_y + rr * std::sin(th);
        }
    }

    auto upload = [&](void *dst, const void *src, size_t bytes) -> int {
        HIPCHK(h, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream));
        return LBM_OK;
    };
    if ((rc = upload(h->runs_dev, h->runs.data(), sizeof(RunDev) * n_runs)) || (rc = build_tiles(h))) {
        g_create_error = h->err;
        delete h;
        return rc;
    }
    std::vector<std::vector<unsigned char>> qtabs(n_runs);
    for (int r = 0; r < n_runs; ++r) {
        qtabs[r] = cut_link_table(h->runs[r], prec);
        if (!qtabs[r].empty() && (rc = upload((void *)h->runs[r].qtab, qtabs[r].data(), qtabs[r].size()))) {
            g_create_error = h->err;
            delete h;
            return rc;
        }
        if ((rc = upload((void *)h->runs[r].probes, probes[r].data(), sizeof(double) * probes[r].size()))) {
            g_create_error = h->err;
            delete h;
            return rc;
        }
    }
    // diagnostic workgroups: rows of each run in order
    std::vector<lbm::DiagBlock> dblocks;
    for (int r = 0; r < n_runs; ++r) {
        const int rows = diag_rows(cfgs[r]);
        h->diag_off.push_back((int)dblocks.size());
        for (int b = 0, y = 0; y < cfgs[r].ny; ++b, y += rows)
            dblocks.push_back(lbm::DiagBlock{r, y, std::min(cfgs[r].ny, y + rows), b});
        h->diag_cnt.push_back((int)dblocks.size() - h->diag_off.back());
    }
    if ((rc = upload(h->diag_blocks, dblocks.data(), sizeof(lbm::DiagBlock) * dblocks.size()))) {
        g_create_error = h->err;
        delete h;
        return rc;
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        delete h;
        return fail(nullptr, LBM_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    // default state of every run: saturated liquid moving with the inlet velocity at T_sat
    for (int r = 0; r < n_runs; ++r) {
        const RunDev &R = h->runs[r];
        std::vector<double> rho((size_t)R.nx * R.ny, R.rho_l), ux(rho.size(), R.bc_x == 1 ? cfgs[r].u_in : 0.0),
            uy(rho.size(), 0.0);
        const int seed = prec == LBM_F64_TANGENT && R.bc_x == 1 ? 1 : -1;  // d(u)/d(u_in) = 1
        if ((rc = set_fields_impl(h, r, rho.data(), ux.data(), uy.data(), nullptr, seed)) != LBM_OK) {
            g_create_error = h->err;
            delete h;
            return rc;
        }
    }
    h->default_state.assign(n_runs, 1);
    *out = h;
    return LBM_OK;
}

int lbm_set_fields(lbm_handle *h, int run, const double *rho, const double *ux, const double *uy, const double *T)
{
    return set_fields_impl(h, run, rho, ux, uy, T, -1);
}

// ux_seed_dir >= 0 (tangent precision): the x velocity field is the inlet velocity, so its
// derivative along that direction is 1
static int set_fields_impl(lbm_handle *h, int run, const double *rho, const double *ux, const double *uy,
                           const double *T, int ux_seed_dir)
{
    int rc = check_run(h, run);
    if (rc) return rc;
    if (!rho || !ux || !uy) return fail(h, LBM_EINVAL, "rho, ux and uy are required");
    // make the target buffers the current ones of every run: bring other runs along by copying
    if (h->pf != 0 || h->pt != 0 || h->ph != 0) {
        for (int r = 0; r < h->n_runs; ++r) {
            const RunDev &R = h->runs[r];
            const size_t plane = (size_t)R.ny * R.pitch;
            if (h->pf) HIPCHK(h, hipMemcpyAsync(R.f[0], R.f[1], 9 * plane * storage_bytes(h->precision), hipMemcpyDeviceToDevice, h->stream));
            if (h->pt) HIPCHK(h, hipMemcpyAsync(R.T[0], R.T[1], plane * compute_bytes(h->precision), hipMemcpyDeviceToDevice, h->stream));
            if (h->ph) HIPCHK(h, hipMemcpyAsync(R.hist[0], R.hist[1], 3 * (size_t)R.ny * compute_bytes(h->precision), hipMemcpyDeviceToDevice, h->stream));
        }
        h->pf = h->pt = h->ph = 0;
    }
    const RunDev &R = h->runs[run];
    if ((rc = upload_plane(h, R, R.rho, rho, 0)) || (rc = upload_plane(h, R, R.ux, ux, 0, ux_seed_dir)) ||
        (rc = upload_plane(h, R, R.uy, uy, 0)) || (rc = upload_plane(h, R, R.T[0], T, R.T_sat)))
        return rc;
    HIPCHK(h, hipMemsetAsync(R.acc, 0, sizeof(double) * lbm::kAcc, h->stream));
    HIPCHK(h, lbm::launch_init(h->precision, h->runs_dev, run, (long long)R.nx * R.ny, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->step = 0;
    if (run < (int)h->default_state.size()) h->default_state[run] = 0;
    return LBM_OK;
}

// Enqueue the launches of one step (no host synchronisation).  tm (optional, three entries): events
// of the k_lbm dispatch, of the k_thermal dispatch and around the step's diagnostic reductions;
// *thermal_ran / *diag_ran tell whether the latter two were launched.
static int enqueue_step(lbm_handle *h, const lbm::Timing *tm = nullptr, bool *thermal_ran = nullptr,
                        bool *diag_ran = nullptr)
{
    HIPCHK(h, lbm::launch_lbm(h->precision, h->var[0], true, h->phase, h->runs_dev, h->tiles_lbm, h->n_lbm, h->pf, h->pt, h->ph,
                              h->step, h->stream, tm));
    bool thermal = false, diag = false;
    for (int r = 0; r < h->n_runs; ++r) {
        const lbm_config &k = h->cfgs[r];
        const bool fon = h->step >= k.warmup_steps;
        diag |= (k.diag_every > 0 && fon && h->step % k.diag_every == 0) || (k.check_every > 0 && h->step % k.check_every == 0);
        thermal |= fon && k.rk_stages > 0;
    }
    if (diag) {
        // one launch; each run takes part when its sample or check falls on this step
        if (tm) HIPCHK(h, hipEventRecord(tm[2].start, h->stream));
        HIPCHK(h, lbm::launch_diag(h->precision, h->runs_dev, h->diag_blocks, h->diag_off.back() + h->diag_cnt.back(), 0,
                                   h->n_runs, h->pt, h->step, -1, h->stream));
        if (tm) HIPCHK(h, hipEventRecord(tm[2].stop, h->stream));
    }
    if (thermal) {
        HIPCHK(h, lbm::launch_thermal(h->precision, h->rk, h->var[1], h->phase, h->runs_dev, h->tiles_th, h->n_th, h->pt, h->step,
                                      h->stream, tm ? tm + 1 : nullptr));
        h->pt ^= 1;
    }
    if (thermal_ran) *thermal_ran = thermal;
    if (diag_ran) *diag_ran = diag;
    std::fill(h->default_state.begin(), h->default_state.end(), 0);
    h->pf ^= 1;
    h->ph ^= 1;
    h->step += 1;
    return LBM_OK;
}

// One step of every run, group by group on the groups' streams (same launches and order per run
// as enqueue_step; the tiles of a group's runs are contiguous in the tile tables).
static int enqueue_step_groups(lbm_handle *h)
{
    bool thermal = false;
    for (int r = 0; r < h->n_runs; ++r)
        thermal |= h->step >= h->cfgs[r].warmup_steps && h->cfgs[r].rk_stages > 0;
    for (const auto &g : h->groups) {
        const int l0 = h->lbm_off[g.run0], l1 = h->lbm_off[g.run1 - 1] + h->lbm_cnt[g.run1 - 1];
        HIPCHK(h, lbm::launch_lbm(h->precision, h->var[0], true, h->phase, h->runs_dev, h->tiles_lbm + l0, l1 - l0, h->pf,
                                  h->pt, h->ph, h->step, g.s));
        bool diag = false;
        for (int r = g.run0; r < g.run1; ++r) {
            const lbm_config &k = h->cfgs[r];
            const bool fon = h->step >= k.warmup_steps;
            diag |= (k.diag_every > 0 && fon && h->step % k.diag_every == 0) ||
                    (k.check_every > 0 && h->step % k.check_every == 0);
        }
        if (diag) {
            const int d0 = h->diag_off[g.run0], d1 = h->diag_off[g.run1 - 1] + h->diag_cnt[g.run1 - 1];
            HIPCHK(h, lbm::launch_diag(h->precision, h->runs_dev, h->diag_blocks + d0, d1 - d0, g.run0, g.run1 - g.run0, h->pt,
                                       h->step, -1, g.s));
        }
        if (thermal) {
            const int t0 = h->th_off[g.run0], t1 = h->th_off[g.run1 - 1] + h->th_cnt[g.run1 - 1];
            HIPCHK(h, lbm::launch_thermal(h->precision, h->rk, h->var[1], h->phase, h->runs_dev, h->tiles_th + t0, t1 - t0,
                                          h->pt, h->step, g.s));
        }
    }
    if (thermal) h->pt ^= 1;
    std::fill(h->default_state.begin(), h->default_state.end(), 0);
    h->pf ^= 1;
    h->ph ^= 1;
    h->step += 1;
    return LBM_OK;
}

static void drop_groups(lbm_handle *h)
{
    for (auto &g : h->groups) {
        (void)hipStreamSynchronize(g.s);
        (void)hipEventDestroy(g.done);
        (void)hipStreamDestroy(g.s);
    }
    h->groups.clear();
    if (h->fork) (void)hipEventDestroy(h->fork);
    h->fork = nullptr;
}

static long long lcm_ll(long long a, long long b)
{
    long long x = a, y = b;
    while (y) { long long t = x % y; x = y; y = t; }
    return a / x * b;
}

// Length of the repeating launch pattern once every run is past its warm-up: populations and
// outlet history alternate buffers every step, the temperature every step, and the Nu
// accumulation / checks recur with their own periods.
static long long pattern_length(const lbm_handle *h)
{
    long long L = 2;
    for (const auto &k : h->cfgs) {
        if (k.diag_every > 0) L = lcm_ll(L, k.diag_every);
        if (k.check_every > 0) L = lcm_ll(L, k.check_every);
    }
    return L;
}

int lbm_step(lbm_handle *h, int n_steps)
{
    const Range range("lbm_step");
    if (int rc_ = check_handle(h)) return rc_;
    if (n_steps < 0) return fail(h, LBM_EINVAL, "negative step count");
    bool any_check = false;
    int max_warm = 0;
    for (int r = 0; r < h->n_runs; ++r) {
        any_check |= h->cfgs[r].check_every > 0;
        max_warm = std::max(max_warm, h->cfgs[r].warmup_steps);
    }
    const long long L = pattern_length(h);
    const int ng = (int)h->groups.size();
    long long remaining = n_steps;
    // k steps by direct launches: on the caller's stream, or forked from it onto the group streams
    // (every group's runs stepped on its own stream) and joined back
    auto eager_steps = [&](long long k) -> int {
        if (ng == 0) {
            for (long long j = 0; j < k; ++j)
                if (int rc = enqueue_step(h)) return rc;
            return LBM_OK;
        }
        HIPCHK(h, hipEventRecord(h->fork, h->stream));
        for (const auto &g : h->groups) HIPCHK(h, hipStreamWaitEvent(g.s, h->fork, 0));
        for (long long j = 0; j < k; ++j)
            if (int rc = enqueue_step_groups(h)) return rc;
        for (const auto &g : h->groups) {
            HIPCHK(h, hipEventRecord(g.done, g.s));
            HIPCHK(h, hipStreamWaitEvent(h->stream, g.done, 0));
        }
        return LBM_OK;
    };
    while (remaining > 0) {
        // replay a captured window when the pattern repeats (all runs past warm-up, window aligned)
        const bool periodic = h->step >= max_warm;
        if (h->use_graphs && periodic && L <= 4096 && remaining >= L && h->step % L == 0) {
            StepGraph *g = nullptr;
            for (auto &c : h->graphs)
                if (c.pf == h->pf && c.pt == h->pt && c.ph == h->ph && c.length == (int)L && c.groups == ng) g = &c;
            if (!g) {
                StepGraph c{h->pf, h->pt, h->ph, (int)L, ng, h->step, nullptr, nullptr};
                const int pf = h->pf, pt = h->pt, ph = h->ph;
                const long long st = h->step;
                // record on a private stream (the caller's may be the legacy default stream, which
                // cannot be captured); the graph is launched on the caller's stream.  With stream
                // groups the fork and join events bring the group streams into the capture, so the
                // groups become parallel branches of the graph.
                if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
                hipStream_t user = h->stream;
                h->stream = h->cap_stream;
                hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
                int rc = LBM_OK;
                if (e == hipSuccess) {
                    rc = eager_steps(L);
                    hipGraph_t graph = nullptr;
                    const hipError_t e2 = hipStreamEndCapture(h->stream, &graph);
                    c.graph = graph;
                    e = rc == LBM_OK ? e2 : hipSuccess;
                    if (rc != LBM_OK && graph) (void)hipGraphDestroy(graph);
                }
                h->stream = user;
                // the capture only recorded work: restore the counters it advanced
                h->pf = pf; h->pt = pt; h->ph = ph; h->step = st;
                if (rc != LBM_OK) return rc;
                if (e != hipSuccess) return fail(h, LBM_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
                HIPCHK(h, hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0));
                h->graphs.push_back(c);
                g = &h->graphs.back();
            }
            const int pt0 = h->pt;
            long long reps = remaining / L;
            for (long long k = 0; k < reps; ++k) HIPCHK(h, hipGraphLaunch(g->exec, h->stream));
            // parities return to their values after an even-length window
            h->pt = pt0;
            std::fill(h->default_state.begin(), h->default_state.end(), 0);
            h->step += reps * L;
            remaining -= reps * L;
            continue;
        }
        // direct launches until the window is aligned (or without graphs)
        long long eager = remaining;
        if (h->use_graphs && periodic) eager = std::min(eager, L - h->step % L);
        else if (h->use_graphs && !periodic) eager = std::min(eager, (long long)max_warm - h->step);
        if (int rc = eager_steps(eager)) return rc;
        remaining -= eager;
    }
    if (any_check) {
        for (int r = 0; r < h->n_runs; ++r) {
            double acc[lbm::kAcc];
            HIPCHK(h, hipMemcpyAsync(acc, h->runs[r].acc, sizeof(acc), hipMemcpyDeviceToHost, h->stream));
            HIPCHK(h, hipStreamSynchronize(h->stream));
            if (acc[5] != 0.0) return fail(h, LBM_EUNSTABLE, "run %d: non-finite state detected", r);
        }
    }
    return LBM_OK;
}

int lbm_fields(lbm_handle *h, int run, double *rho, double *ux, double *uy, double *T, uint8_t *mask)
{
    const Range range("lbm_fields");
    int rc = check_run(h, run);
    if (rc) return rc;
    const RunDev &R = h->runs[run];
    if ((rc = moments_pass(h, run))) return rc;
    std::vector<double> buf;
    struct { void *src; double *dst; bool zero_solid; } outs[4] = {
        {R.rho, rho, true}, {R.ux, ux, true}, {R.uy, uy, true}, {R.T[h->pt], T, false}};
    for (auto &o : outs) {
        if (!o.dst) continue;
        if ((rc = download_plane(h, R, o.src, buf))) return rc;
        for (int y = 0; y < R.ny; ++y)
            for (int x = 0; x < R.nx; ++x) {
                const size_t k = (size_t)y * R.nx + x;
                o.dst[k] = (o.zero_solid && solid_host(R, x, y)) ? 0.0 : buf[k];
            }
    }
    if (mask)
        for (int y = 0; y < R.ny; ++y)
            for (int x = 0; x < R.nx; ++x) mask[(size_t)y * R.nx + x] = solid_host(R, x, y) ? 1 : 0;
    return LBM_OK;
}

int lbm_get_state(lbm_handle *h, int run, double *fstar, double *hist, double *T)
{
    int rc = check_run(h, run);
    if (rc) return rc;
    const RunDev &R = h->runs[run];
    const size_t plane = (size_t)R.ny * R.pitch;
    if (fstar) {
        const size_t sb = storage_bytes(h->precision);
        std::vector<unsigned char> raw(9 * plane * sb);
        HIPCHK(h, hipMemcpyAsync(raw.data(), R.f[h->pf], raw.size(), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        for (int i = 0; i < 9; ++i)
            for (int y = 0; y < R.ny; ++y)
                for (int x = 0; x < R.nx; ++x) {
                    double v = ld_storage(raw.data(), h->precision, (size_t)i * plane + (size_t)y * R.pitch + x);
                    if (h->precision >= 2) v += (double)(float)(kW[i] * R.shift);
                    fstar[((size_t)i * R.ny + y) * R.nx + x] = v;
                }
    }
    if (hist) {
        const size_t cb = compute_bytes(h->precision);
        std::vector<unsigned char> raw(3 * (size_t)R.ny * cb);
        HIPCHK(h, hipMemcpyAsync(raw.data(), R.hist[h->ph], raw.size(), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        for (size_t k = 0; k < 3 * (size_t)R.ny; ++k) hist[k] = ld_compute(raw.data(), h->precision, k);
    }
    if (T) {
        std::vector<double> buf;
        if ((rc = download_plane(h, R, R.T[h->pt], buf))) return rc;
        std::copy(buf.begin(), buf.end(), T);
    }
    return LBM_OK;
}

int lbm_set_state(lbm_handle *h, int run, const double *fstar, const double *hist, const double *T, int64_t step)
{
    int rc = check_run(h, run);
    if (rc) return rc;
    if (!fstar || !hist || !T) return fail(h, LBM_EINVAL, "fstar, hist and T are required");
    const RunDev &R = h->runs[run];
    const size_t plane = (size_t)R.ny * R.pitch;
    const size_t sb = storage_bytes(h->precision), cb = compute_bytes(h->precision);
    std::vector<unsigned char> raw(9 * plane * sb, 0);
    for (int i = 0; i < 9; ++i)
        for (int y = 0; y < R.ny; ++y)
            for (int x = 0; x < R.nx; ++x) {
                double v = fstar[((size_t)i * R.ny + y) * R.nx + x];
                if (h->precision >= 2) v -= (double)(float)(kW[i] * R.shift);
                st_storage(raw.data(), h->precision, (size_t)i * plane + (size_t)y * R.pitch + x, v);
            }
    HIPCHK(h, hipMemcpyAsync(R.f[h->pf], raw.data(), raw.size(), hipMemcpyHostToDevice, h->stream));
    std::vector<unsigned char> hraw(3 * (size_t)R.ny * cb);
    for (size_t k = 0; k < 3 * (size_t)R.ny; ++k) st_compute(hraw.data(), h->precision, k, hist[k]);
    HIPCHK(h, hipMemcpyAsync(R.hist[h->ph], hraw.data(), hraw.size(), hipMemcpyHostToDevice, h->stream));
    std::vector<double> Tw((size_t)R.nx * R.ny);
    for (int y = 0; y < R.ny; ++y)
        for (int x = 0; x < R.nx; ++x) {
            const size_t k = (size_t)y * R.nx + x;
            Tw[k] = solid_host(R, x, y) ? R.T_w : T[k];
        }
    if ((rc = upload_plane(h, R, R.T[h->pt], Tw.data(), 0))) return rc;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->step = step;
    h->default_state[run] = 0;
    return LBM_OK;
}

}  // extern "C"

namespace {
// Checkpoint layout: a header, then per run the current population buffer (storage format), the
// current outlet history and temperature (compute format) and the FP64 accumulators, byte for byte.
struct CkptHeader {
    char magic[8];
    int32_t n_runs, precision;
    int64_t step;
};
constexpr char kCkptMagic[8] = {'L', 'B', 'M', 'C', 'K', 'P', 'T', '1'};

struct CkptPart {
    void *dev;
    size_t bytes;
};

std::vector<CkptPart> ckpt_parts(const lbm_handle *h)
{
    std::vector<CkptPart> parts;
    const size_t sb = storage_bytes(h->precision), cb = compute_bytes(h->precision);
    for (const RunDev &R : h->runs) {
        const size_t plane = (size_t)R.ny * R.pitch;
        parts.push_back({R.f[h->pf], 9 * plane * sb});
        parts.push_back({R.hist[h->ph], 3 * (size_t)R.ny * cb});
        parts.push_back({R.T[h->pt], plane * cb});
        parts.push_back({R.acc, sizeof(double) * lbm::kAcc});
    }
    return parts;
}

size_t ckpt_bytes(const lbm_handle *h)
{
    size_t b = sizeof(CkptHeader) + sizeof(int32_t) * 2 * (size_t)h->n_runs;
    for (const CkptPart &p : ckpt_parts(h)) b += p.bytes;
    return b;
}
}  // namespace

extern "C" {

size_t lbm_checkpoint_bytes(const lbm_handle *h) { return h ? ckpt_bytes(h) : 0; }

int lbm_save(lbm_handle *h, void *host_buf, size_t bytes)
{
    const Range range("lbm_save");
    if (int rc_ = check_handle(h)) return rc_;
    if (!host_buf) return fail(h, LBM_EINVAL, "host_buf is NULL");
    if (bytes < ckpt_bytes(h)) return fail(h, LBM_EINVAL, "checkpoint needs %zu bytes", ckpt_bytes(h));
    unsigned char *p = (unsigned char *)host_buf;
    CkptHeader hd;
    std::memcpy(hd.magic, kCkptMagic, sizeof(hd.magic));
    hd.n_runs = h->n_runs;
    hd.precision = h->precision;
    hd.step = h->step;
    std::memcpy(p, &hd, sizeof(hd));
    p += sizeof(hd);
    for (const auto &c : h->cfgs) {
        const int32_t g[2] = {c.nx, c.ny};
        std::memcpy(p, g, sizeof(g));
        p += sizeof(g);
    }
    for (const CkptPart &part : ckpt_parts(h)) {
        HIPCHK(h, hipMemcpyAsync(p, part.dev, part.bytes, hipMemcpyDeviceToHost, h->stream));
        p += part.bytes;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_load(lbm_handle *h, const void *host_buf, size_t bytes)
{
    const Range range("lbm_load");
    if (int rc_ = check_handle(h)) return rc_;
    if (!host_buf) return fail(h, LBM_EINVAL, "host_buf is NULL");
    if (bytes < ckpt_bytes(h)) return fail(h, LBM_EINVAL, "checkpoint of %zu bytes, this handle's take %zu", bytes, ckpt_bytes(h));
    const unsigned char *p = (const unsigned char *)host_buf;
    CkptHeader hd;
    std::memcpy(&hd, p, sizeof(hd));
    p += sizeof(hd);
    if (std::memcmp(hd.magic, kCkptMagic, sizeof(hd.magic)) != 0) return fail(h, LBM_EINVAL, "not a checkpoint");
    if (hd.n_runs != h->n_runs || hd.precision != h->precision)
        return fail(h, LBM_EINVAL, "checkpoint of %d runs in precision %d, handle has %d runs in precision %d", hd.n_runs,
                    hd.precision, h->n_runs, h->precision);
    for (const auto &c : h->cfgs) {
        int32_t g[2];
        std::memcpy(g, p, sizeof(g));
        p += sizeof(g);
        if (g[0] != c.nx || g[1] != c.ny) return fail(h, LBM_EINVAL, "checkpoint grid %dx%d differs from %dx%d", g[0], g[1], c.nx, c.ny);
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (const CkptPart &part : ckpt_parts(h)) {
        HIPCHK(h, hipMemcpyAsync(part.dev, p, part.bytes, hipMemcpyHostToDevice, h->stream));
        p += part.bytes;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->step = hd.step;
    std::fill(h->default_state.begin(), h->default_state.end(), 0);
    drop_graphs(h);
    return LBM_OK;
}

int lbm_wall_heat_flux(lbm_handle *h, int run, double *q_mean, double *nu, double *nu_time_avg)
{
    const Range range("lbm_wall_heat_flux");
    int rc = check_run(h, run);
    if (rc) return rc;
    if ((rc = moments_pass(h, run))) return rc;
    HIPCHK(h, lbm::launch_diag(h->precision, h->runs_dev, h->diag_blocks + h->diag_off[run], h->diag_cnt[run], run, 1,
                               h->pt, h->step, run, h->stream));
    double acc[8];
    HIPCHK(h, hipMemcpyAsync(acc, h->runs[run].acc, sizeof(acc), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (q_mean) *q_mean = acc[1];
    if (nu) *nu = acc[2];
    if (nu_time_avg) *nu_time_avg = acc[4] > 0 ? acc[3] / acc[4] : 0.0;
    return LBM_OK;
}

int lbm_nu_tangent(lbm_handle *h, int run, double *dnu, double *dnu_time_avg)
{
    int rc = check_run(h, run);
    if (rc) return rc;
    if (h->precision != LBM_F64_TANGENT) return fail(h, LBM_EINVAL, "the handle does not carry tangents");
    if ((rc = moments_pass(h, run))) return rc;
    HIPCHK(h, lbm::launch_diag(h->precision, h->runs_dev, h->diag_blocks + h->diag_off[run], h->diag_cnt[run], run, 1,
                               h->pt, h->step, run, h->stream));
    double acc[lbm::kAcc];
    HIPCHK(h, hipMemcpyAsync(acc, h->runs[run].acc, sizeof(acc), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int k = 0; k < lbm::kTangents; ++k) {
        if (dnu) dnu[k] = acc[8 + k];
        if (dnu_time_avg) dnu_time_avg[k] = acc[4] > 0 ? acc[12 + k] / acc[4] : 0.0;
    }
    return LBM_OK;
}

int lbm_reset_time_average(lbm_handle *h, int run)
{
    int rc = check_run(h, run);
    if (rc) return rc;
    double acc[lbm::kAcc];
    HIPCHK(h, hipMemcpyAsync(acc, h->runs[run].acc, sizeof(acc), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    acc[3] = acc[4] = 0.0;
    for (int k = 0; k < lbm::kTangents; ++k) acc[12 + k] = 0.0;
    HIPCHK(h, hipMemcpyAsync(h->runs[run].acc, acc, sizeof(acc), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_total_mass(lbm_handle *h, int run, double *mass)
{
    int rc = check_run(h, run);
    if (rc) return rc;
    if ((rc = moments_pass(h, run))) return rc;
    HIPCHK(h, lbm::launch_diag(h->precision, h->runs_dev, h->diag_blocks + h->diag_off[run], h->diag_cnt[run], run, 1,
                               h->pt, h->step, run, h->stream));
    double acc[8];
    HIPCHK(h, hipMemcpyAsync(acc, h->runs[run].acc, sizeof(acc), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (mass) *mass = acc[0];
    return LBM_OK;
}

int lbm_saturation(const lbm_config *cfg, double *out6)
{
    if (!cfg || !out6) return fail(nullptr, LBM_EINVAL, "NULL argument");
    if (!(cfg->eos_a > 0) || !(cfg->eos_b > 0) || !(cfg->eos_R > 0) || !(cfg->Tr_sat > 0 && cfg->Tr_sat < 1))
        return fail(nullptr, LBM_EINVAL, "EOS constants out of range");
    const PR pr(*cfg);
    const double T = cfg->Tr_sat * pr.Tc;
    double rv, rl;
    if (!maxwell(pr, T, rv, rl)) return fail(nullptr, LBM_EINVAL, "no liquid-vapour coexistence at T_sat");
    const double vl = 1.0 / rl, vv = 1.0 / rv, b = pr.b, s2 = std::sqrt(2.0);
    // h_fg = T (s_v - s_l) with s_v - s_l = int_{v_l}^{v_v} (dp/dT)_v dv (a Maxwell relation), and
    // (dp/dT)_v = R/(v - b) - a phi'(T)/(v^2 + 2bv - b^2), phi'(T) = -kappa (1 + kappa (1 - sqrt(T/Tc))) / sqrt(T Tc)
    const double dphi = -pr.kappa * (1.0 + pr.kappa * (1.0 - std::sqrt(T / pr.Tc))) / std::sqrt(T * pr.Tc);
    auto I = [&](double v) { return std::log((v + b - s2 * b) / (v + b + s2 * b)) / (2.0 * s2 * b); };
    const double ds = pr.R * std::log((vv - b) / (vl - b)) - pr.a * dphi * (I(vv) - I(vl));
    out6[0] = pr.Tc;
    out6[1] = T;
    out6[2] = pr.p_v(vv, T);
    out6[3] = rl;
    out6[4] = rv;
    out6[5] = T * ds;
    return LBM_OK;
}

int lbm_derived(lbm_handle *h, int run, double *out8)
{
    int rc = check_run(h, run);
    if (rc) return rc;
    if (!out8) return fail(h, LBM_EINVAL, "out8 is NULL");
    const RunDev &R = h->runs[run];
    const double v[8] = {R.Tc, R.T_sat, R.T_w, R.rho_l, R.rho_v, R.rho_w, R.rho_gref, R.omega};
    std::memcpy(out8, v, sizeof(v));
    return LBM_OK;
}

int lbm_time_kernel(lbm_handle *h, int kernel, int n_launches)
{
    if (int rc_ = check_handle(h)) return rc_;
    if (n_launches < 0) return fail(h, LBM_EINVAL, "negative launch count");
    if (kernel == LBM_KERNEL_STREAM_COLLIDE) {
        for (int k = 0; k < n_launches; ++k)
            HIPCHK(h, lbm::launch_lbm(h->precision, h->var[0], true, h->phase, h->runs_dev, h->tiles_lbm, h->n_lbm, h->pf, h->pt,
                                      h->ph, h->step, h->stream));
        return LBM_OK;
    }
    if (kernel == LBM_KERNEL_THERMAL) {
        if (h->rk == 0) return fail(h, LBM_EINVAL, "runs have no temperature update");
        for (int k = 0; k < n_launches; ++k)
            HIPCHK(h, lbm::launch_thermal(h->precision, h->rk, h->var[1], h->phase, h->runs_dev, h->tiles_th, h->n_th, h->pt,
                                          std::max<long long>(h->step, max_warmup(h)), h->stream));
        return LBM_OK;
    }
    return fail(h, LBM_EINVAL, "unknown kernel %d", kernel);
}

}  // extern "C"

namespace {
// events of a profiled step sequence, released on every return path
struct EventPool {
    std::vector<hipEvent_t> ev;
    ~EventPool()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};
}  // namespace

extern "C" {

int lbm_profile_steps(lbm_handle *h, int n_steps, double *kernel_ms)
{
    const Range range("lbm_profile_steps");
    if (int rc_ = check_handle(h)) return rc_;
    if (!kernel_ms) return fail(h, LBM_EINVAL, "kernel_ms is NULL");
    if (n_steps < 1 || n_steps > LBM_MAX_PROFILE_STEPS)
        return fail(h, LBM_EINVAL, "profiled step count %d outside [1, %d]", n_steps, LBM_MAX_PROFILE_STEPS);
    EventPool pool;
    pool.ev.reserve((size_t)6 * n_steps);
    for (int k = 0; k < 6 * n_steps; ++k) {
        hipEvent_t e;
        HIPCHK(h, hipEventCreate(&e));
        pool.ev.push_back(e);
    }
    std::vector<char> ran((size_t)2 * n_steps, 0);
    for (int s = 0; s < n_steps; ++s) {
        const lbm::Timing tm[3] = {{pool.ev[6 * s], pool.ev[6 * s + 1]}, {pool.ev[6 * s + 2], pool.ev[6 * s + 3]},
                                   {pool.ev[6 * s + 4], pool.ev[6 * s + 5]}};
        bool th = false, dg = false;
        const int rc = enqueue_step(h, tm, &th, &dg);
        if (rc) return rc;
        ran[2 * s] = th;
        ran[2 * s + 1] = dg;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    double sum[3] = {0, 0, 0};
    int cnt[2] = {0, 0};
    for (int s = 0; s < n_steps; ++s)
        for (int k = 0; k < 3; ++k) {
            if (k >= 1 && !ran[2 * s + (k - 1)]) continue;
            float ms = 0;
            HIPCHK(h, hipEventElapsedTime(&ms, pool.ev[6 * s + 2 * k], pool.ev[6 * s + 2 * k + 1]));
            sum[k] += ms;
            if (k < 2) cnt[k] += 1;
        }
    for (int k = 0; k < 2; ++k) kernel_ms[k] = cnt[k] ? sum[k] / cnt[k] : 0.0;
    kernel_ms[2] = sum[2] / n_steps;
    return LBM_OK;
}

int lbm_variant_count(int precision, int kernel)
{
    if (precision < 0 || precision > 3 || kernel < 0 || kernel > 1) return 0;
    return lbm::variant_count(precision, kernel);
}

int lbm_variant_shape(int precision, int kernel, int variant, int *tx, int *ty, int *threads, int *min_waves)
{
    const lbm::Variant v = lbm::variant_shape(precision, kernel, variant);
    if (v.tx == 0) return LBM_EINVAL;
    if (tx) *tx = v.tx;
    if (ty) *ty = v.ty;
    if (threads) *threads = v.nt;
    if (min_waves) *min_waves = v.min_waves;
    return LBM_OK;
}

int lbm_set_variant(lbm_handle *h, int kernel, int variant)
{
    if (int rc_ = check_handle(h)) return rc_;
    if (kernel < 0 || kernel > 1 || variant < 0 || variant >= lbm::variant_count(h->precision, kernel))
        return fail(h, LBM_EINVAL, "no variant %d of kernel %d", variant, kernel);
    const int old = h->var[kernel];
    h->var[kernel] = variant;
    int rc = build_tiles(h);
    if (rc) h->var[kernel] = old;
    return rc;
}

int lbm_get_variant(const lbm_handle *h, int kernel)
{
    if (!h || kernel < 0 || kernel > 1) return -1;
    return h->var[kernel];
}

}  // extern "C"

namespace {
// Tuned launch variants of this process, per device and workload shape: precision, RK stages, the
// extended-feature launch, and every run's grid, cylinder radius and x boundary.
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune_cache;

std::string tune_key(const lbm_handle *h)
{
    int dev = -1;
    (void)hipGetDevice(&dev);
    std::string k = std::to_string(dev) + "/" + std::to_string(h->precision) + "/" + std::to_string(h->rk) + "/" +
                    std::to_string(h->phase ? 1 : 0);
    for (const auto &c : h->cfgs)
        k += "/" + std::to_string(c.nx) + "x" + std::to_string(c.ny) + "r" + std::to_string(c.cyl_r) + "b" +
             std::to_string(c.bc_x);
    return k;
}
}  // namespace

extern "C" {

// n pseudo-steps on the current state without advancing it: the stream-and-collide kernel (writing
// the spare population buffer and the macroscopic fields) and the temperature update (reading those
// fields, writing the spare temperature buffer) in turn, as in a step, so that each is timed with
// the caches the other leaves behind
static int time_pseudo_steps(lbm_handle *h, int n)
{
    const long long th_step = std::max<long long>(h->step, max_warmup(h));
    for (int k = 0; k < n; ++k) {
        HIPCHK(h, lbm::launch_lbm(h->precision, h->var[0], true, h->phase, h->runs_dev, h->tiles_lbm, h->n_lbm, h->pf,
                                  h->pt, h->ph, h->step, h->stream));
        if (h->rk != 0)
            HIPCHK(h, lbm::launch_thermal(h->precision, h->rk, h->var[1], h->phase, h->runs_dev, h->tiles_th, h->n_th,
                                          h->pt, th_step, h->stream));
    }
    return LBM_OK;
}

int lbm_autotune(lbm_handle *h, int launches, int *best)
{
    const Range range("lbm_autotune");
    if (int rc_ = check_handle(h)) return rc_;
    const std::string key = tune_key(h);
    if (launches < 0) {
        std::pair<int, int> hit(-1, -1);
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) hit = it->second;
        }
        if (hit.first >= 0) {
            int rc = lbm_set_variant(h, 0, hit.first);
            if (!rc && h->rk != 0) rc = lbm_set_variant(h, 1, hit.second);
            if (rc) return rc;
            if (best) { best[0] = h->var[0]; best[1] = h->var[1]; }
            return LBM_OK;
        }
    }
    if (launches <= 0) launches = 20;
    // the launches timed: whole steps of the handle (the state advances), or pseudo-steps that
    // leave it as it is
    auto timed = [&](int n) -> int {
        if (!h->tune_steps) return time_pseudo_steps(h, n);
        for (int j = 0; j < n; ++j)
            if (int rc = enqueue_step(h)) return rc;
        return LBM_OK;
    };
    EventPool pool;  // released on every return path
    for (int k = 0; k < 2; ++k) {
        hipEvent_t e;
        HIPCHK(h, hipEventCreate(&e));
        pool.ev.push_back(e);
    }
    hipEvent_t e0 = pool.ev[0], e1 = pool.ev[1];
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && h->rk == 0) continue;
        // two interleaved rounds over the variants of kernel k (the other kernel at its current
        // variant), each timed over the launches above; each variant keeps its faster round
        const int nv = lbm::variant_count(h->precision, k);
        std::vector<float> t(nv, 1e30f);
        for (int round = 0; round < 2; ++round)
            for (int v = 0; v < nv; ++v) {
                int rc = lbm_set_variant(h, k, v);
                if (rc) return rc;
                if ((rc = timed(3))) return rc;
                HIPCHK(h, hipEventRecord(e0, h->stream));
                if ((rc = timed(launches))) return rc;
                HIPCHK(h, hipEventRecord(e1, h->stream));
                HIPCHK(h, hipEventSynchronize(e1));
                float ms = 0;
                HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
                t[v] = std::min(t[v], ms);
            }
        int best_v = h->var[k];
        float best_ms = 1e30f;
        for (int v = 0; v < nv; ++v)
            if (t[v] < best_ms) { best_ms = t[v]; best_v = v; }
        int rc = lbm_set_variant(h, k, best_v);
        if (rc) return rc;
        if (best) best[k] = best_v;
    }
    if (best && h->rk == 0) best[1] = h->var[1];
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = std::make_pair(h->var[0], h->var[1]);
    return LBM_OK;
}

int lbm_set_option(lbm_handle *h, int option, int value)
{
    if (int rc_ = check_handle(h)) return rc_;
    if (option == LBM_OPT_GRAPHS) {
        h->use_graphs = value != 0;
        drop_graphs(h);
        return LBM_OK;
    }
    if (option == LBM_OPT_TUNE_STEPS) {
        if (value != 0 && value != 1) return fail(h, LBM_EINVAL, "LBM_OPT_TUNE_STEPS takes 0 or 1");
        h->tune_steps = value != 0;
        return LBM_OK;
    }
    if (option == LBM_OPT_STREAM_GROUPS) {
        if (value < 1 || value > LBM_MAX_STREAM_GROUPS || value > h->n_runs)
            return fail(h, LBM_EINVAL, "stream groups %d outside [1, min(%d, runs = %d)]", value, LBM_MAX_STREAM_GROUPS,
                        h->n_runs);
        HIPCHK(h, hipStreamSynchronize(h->stream));
        drop_groups(h);
        drop_graphs(h);  // windows captured with the former groups
        if (value == 1) return LBM_OK;
        // contiguous ranges of runs with about equal node counts
        std::vector<double> cum(h->n_runs + 1, 0.0);
        for (int r = 0; r < h->n_runs; ++r) cum[r + 1] = cum[r] + (double)h->cfgs[r].nx * h->cfgs[r].ny;
        int r0 = 0;
        for (int g = 0; g < value; ++g) {
            int r1 = r0 + 1;
            const double target = cum[h->n_runs] * (g + 1) / value;
            while (r1 < h->n_runs - (value - 1 - g) && cum[r1] + 0.5 * (cum[r1 + 1] - cum[r1]) < target) ++r1;
            if (g == value - 1) r1 = h->n_runs;
            lbm_handle::Group grp{r0, r1, nullptr, nullptr};
            hipError_t e = hipStreamCreateWithFlags(&grp.s, hipStreamNonBlocking);
            if (e == hipSuccess) {
                e = hipEventCreateWithFlags(&grp.done, hipEventDisableTiming);
                if (e != hipSuccess) (void)hipStreamDestroy(grp.s);
            }
            if (e != hipSuccess) {
                drop_groups(h);
                return fail(h, LBM_EDEVICE, "stream group: %s", hipGetErrorString(e));
            }
            h->groups.push_back(grp);
            r0 = r1;
        }
        hipError_t e = hipEventCreateWithFlags(&h->fork, hipEventDisableTiming);
        if (e != hipSuccess) {
            drop_groups(h);
            return fail(h, LBM_EDEVICE, "stream group: %s", hipGetErrorString(e));
        }
        return LBM_OK;
    }
    return fail(h, LBM_EINVAL, "unknown option %d", option);
}

int lbm_get_option(const lbm_handle *h, int option)
{
    if (!h) return -1;
    if (option == LBM_OPT_GRAPHS) return h->use_graphs ? 1 : 0;
    if (option == LBM_OPT_TUNE_STEPS) return h->tune_steps ? 1 : 0;
    if (option == LBM_OPT_STREAM_GROUPS) return h->groups.empty() ? 1 : (int)h->groups.size();
    return -1;
}

int lbm_stream_group_runs(const lbm_handle *h, int group, int *run0, int *run1)
{
    if (!h) return LBM_EINVAL;
    const int n = h->groups.empty() ? 1 : (int)h->groups.size();
    if (group < 0 || group >= n) return LBM_EINVAL;
    if (run0) *run0 = h->groups.empty() ? 0 : h->groups[group].run0;
    if (run1) *run1 = h->groups.empty() ? h->n_runs : h->groups[group].run1;
    return LBM_OK;
}

}  // extern "C"

namespace {
// the adjoint covers FP64 runs with x periodic or a velocity inlet / convective outlet at speed u_in,
// constant transport properties and grids of at least 5 x 5
int adjoint_supported(lbm_handle *h, int run)
{
    const lbm_config &k = h->cfgs[run];
    if (h->precision != LBM_FP64) return fail(h, LBM_EINVAL, "the adjoint needs an FP64 handle");
    if (k.bc_x != LBM_BC_PERIODIC && k.bc_x != LBM_BC_INLET_OUTLET)
        return fail(h, LBM_EINVAL, "the adjoint covers periodic and inlet/outlet channels only");
    if (h->runs[run].phase_props || k.outlet_kind != LBM_OUTLET_U_IN)
        return fail(h, LBM_EINVAL, "the adjoint covers constant transport properties and the outlet speed u_in only");
    if (k.nx < 5 || k.ny < 5) return fail(h, LBM_EINVAL, "the adjoint needs nx, ny >= 5");
    return LBM_OK;
}

size_t adj_state_bytes(const RunDev &R) { return sizeof(double) * lbm::adjoint_state_doubles(R.nx, R.ny, R.pitch); }

// change a run's Nu sampling period (host launch pattern and the device descriptor)
int set_run_diag(lbm_handle *h, int run, int every)
{
    h->cfgs[run].diag_every = every;
    h->runs[run].diag_every = every;
    HIPCHK(h, hipMemcpyAsync(h->runs_dev + run, &h->runs[run], sizeof(RunDev), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    drop_graphs(h);
    return LBM_OK;
}
size_t adj_scratch_bytes(const RunDev &R) { return sizeof(double) * lbm::adjoint_scratch_doubles(R.nx, R.ny, R.pitch); }
// raw FP64 state of a run in a device slot: f* [9] planes, T plane, outlet history [3][ny]
size_t state_doubles(const RunDev &R) { return 10 * (size_t)R.ny * R.pitch + 3 * (size_t)R.ny; }

int copy_state(lbm_handle *h, int run, double *slot, bool out)
{
    const RunDev &R = h->runs[run];
    const size_t P = (size_t)R.ny * R.pitch;
    struct { void *dev; double *sl; size_t n; } parts[3] = {
        {R.f[h->pf], slot, 9 * P}, {R.T[h->pt], slot + 9 * P, P}, {R.hist[h->ph], slot + 10 * P, 3 * (size_t)R.ny}};
    for (auto &p : parts) {
        if (out) HIPCHK(h, hipMemcpyAsync(p.sl, p.dev, sizeof(double) * p.n, hipMemcpyDeviceToDevice, h->stream));
        else HIPCHK(h, hipMemcpyAsync(p.dev, p.sl, sizeof(double) * p.n, hipMemcpyDeviceToDevice, h->stream));
    }
    return LBM_OK;
}

size_t gradient_bytes(const RunDev &R, int steps, int every)
{
    const size_t nck = (size_t)((steps + every - 1) / every);
    const size_t sd = align256(sizeof(double) * state_doubles(R));
    return (nck + (size_t)every + 1) * sd + 2 * align256(adj_state_bytes(R)) + align256(adj_scratch_bytes(R));
}
}  // namespace

extern "C" {

size_t lbm_adjoint_state_bytes(lbm_handle *h, int run)
{
    if (check_run(h, run) || adjoint_supported(h, run)) return 0;
    return adj_state_bytes(h->runs[run]);
}

size_t lbm_adjoint_scratch_bytes(lbm_handle *h, int run)
{
    if (check_run(h, run) || adjoint_supported(h, run)) return 0;
    return adj_scratch_bytes(h->runs[run]);
}

int lbm_adjoint_step(lbm_handle *h, int run, double nu_weight, const void *adj_in, void *adj_out, void *scratch,
                     size_t scratch_bytes, double *dJ_dparams)
{
    const Range range("lbm_adjoint_step");
    int rc = check_run(h, run);
    if (rc || (rc = adjoint_supported(h, run))) return rc;
    const RunDev &R = h->runs[run];
    if (!adj_in || !adj_out || adj_in == adj_out) return fail(h, LBM_EINVAL, "adj_in and adj_out must be distinct device buffers");
    if (!scratch || scratch_bytes < adj_scratch_bytes(R))
        return fail(h, LBM_ENOMEM, "the adjoint step needs %zu bytes of scratch", adj_scratch_bytes(R));
    HIPCHK(h, lbm::launch_adjoint_step(h->runs_dev, run, R, (const double *)R.f[h->pf], (const double *)R.hist[h->ph],
                                       (const double *)R.T[h->pt], (const double *)adj_in, (double *)adj_out,
                                       (double *)scratch, h->step, nu_weight, h->stream));
    if (dJ_dparams) {
        HIPCHK(h, hipMemcpyAsync(dJ_dparams, (const double *)adj_out + (adj_state_bytes(R) / sizeof(double) - lbm::kTangents),
                                 sizeof(double) * lbm::kTangents, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    return LBM_OK;
}

size_t lbm_nu_gradient_bytes(lbm_handle *h, int steps, int checkpoint_every)
{
    if (check_handle(h) || h->n_runs != 1 || adjoint_supported(h, 0) || steps < 1 || checkpoint_every < 1) return 0;
    return gradient_bytes(h->runs[0], steps, checkpoint_every);
}

int lbm_nu_gradient(lbm_handle *h, int steps, int average_from, int checkpoint_every, void *dev_ws, size_t ws_bytes,
                    double *J, double *dJ_dparams)
{
    const Range range("lbm_nu_gradient");
    int rc = check_handle(h);
    if (rc) return rc;
    if (h->n_runs != 1) return fail(h, LBM_EINVAL, "the Nu gradient takes a handle of one run");
    if ((rc = adjoint_supported(h, 0))) return rc;
    if (steps < 1 || average_from < 0 || average_from >= steps || checkpoint_every < 1)
        return fail(h, LBM_EINVAL, "need steps >= 1, 0 <= average_from < steps, checkpoint_every >= 1");
    if (h->runs[0].np == 0) return fail(h, LBM_EINVAL, "the run has no cylinder (no wall Nusselt number)");
    const RunDev &R = h->runs[0];
    const int K = checkpoint_every;
    if (!dev_ws || ws_bytes < gradient_bytes(R, steps, K))
        return fail(h, LBM_ENOMEM, "the Nu gradient needs %zu bytes of device workspace", gradient_bytes(R, steps, K));
    if (((uintptr_t)dev_ws & 255) != 0) return fail(h, LBM_EINVAL, "the workspace must be 256-byte aligned");
    const int nck = (steps + K - 1) / K;
    const size_t sd = align256(sizeof(double) * state_doubles(R)) / sizeof(double);
    const size_t ad = align256(adj_state_bytes(R)) / sizeof(double);
    double *ckpt = (double *)dev_ws, *store = ckpt + (size_t)nck * sd, *fin = store + (size_t)K * sd;
    double *adj[2] = {fin + sd, fin + sd + ad};
    double *scr = adj[1] + ad;
    const bool deflt = h->default_state[0] != 0;
    const long long n0 = h->step;
    const int diag0 = h->cfgs[0].diag_every;
    auto finish = [&](int code) {
        const int rc2 = set_run_diag(h, 0, diag0);
        return code ? code : rc2;
    };
    // forward: checkpoints every K steps, Nu sampled every step of the averaging window
    if ((rc = set_run_diag(h, 0, 1))) return finish(rc);
    for (int c = 0; c < nck; ++c) {
        const int s0 = c * K, s1 = std::min(steps, s0 + K);
        if ((rc = copy_state(h, 0, ckpt + (size_t)c * sd, true))) return finish(rc);
        if (average_from >= s0 && average_from < s1) {
            if ((rc = lbm_step(h, average_from - s0)) || (rc = lbm_reset_time_average(h, 0)) ||
                (rc = lbm_step(h, s1 - average_from)))
                return finish(rc);
        } else if ((rc = lbm_step(h, s1 - s0))) {
            return finish(rc);
        }
    }
    double acc[lbm::kAcc];
    HIPCHK(h, hipMemcpyAsync(acc, R.acc, sizeof(acc), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const double samples = acc[4];
    if (J) *J = samples > 0 ? acc[3] / samples : 0.0;
    if ((rc = copy_state(h, 0, fin, true))) return finish(rc);
    // reverse sweep over the segments, each recomputed from its checkpoint
    if ((rc = set_run_diag(h, 0, 0))) return finish(rc);
    HIPCHK(h, hipMemsetAsync(adj[0], 0, sizeof(double) * ad, h->stream));
    int cur = 0;
    for (int c = nck - 1; c >= 0; --c) {
        const int s0 = c * K, s1 = std::min(steps, s0 + K);
        if ((rc = copy_state(h, 0, ckpt + (size_t)c * sd, false))) return finish(rc);
        h->step = n0 + s0;
        for (int s = s0; s < s1; ++s) {
            if ((rc = copy_state(h, 0, store + (size_t)(s - s0) * sd, true))) return finish(rc);
            if ((rc = enqueue_step(h))) return finish(rc);
        }
        for (int s = s1 - 1; s >= s0; --s) {
            const long long n = n0 + s;
            const double w = (s >= average_from && n >= h->cfgs[0].warmup_steps && samples > 0) ? 1.0 / samples : 0.0;
            const double *st = store + (size_t)(s - s0) * sd;
            const size_t P = (size_t)R.ny * R.pitch;
            HIPCHK(h, lbm::launch_adjoint_step(h->runs_dev, 0, R, st, st + 10 * P, st + 9 * P, adj[cur], adj[cur ^ 1], scr, n, w,
                                               h->stream));
            cur ^= 1;
        }
    }
    HIPCHK(h, lbm::launch_adjoint_initial(h->runs_dev, 0, adj[cur], deflt, h->stream));
    double g[lbm::kTangents];
    HIPCHK(h, hipMemcpyAsync(g, adj[cur] + (adj_state_bytes(R) / sizeof(double) - lbm::kTangents), sizeof(g),
                             hipMemcpyDeviceToHost, h->stream));
    // the handle ends in the forward run's final state
    if ((rc = copy_state(h, 0, fin, false))) return finish(rc);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->step = n0 + steps;
    if (dJ_dparams) std::memcpy(dJ_dparams, g, sizeof(g));
    return finish(LBM_OK);
}

int64_t lbm_step_count(const lbm_handle *h) { return h ? h->step : -1; }

const char *lbm_last_error(const lbm_handle *h) { return h ? h->err.c_str() : g_create_error.c_str(); }

void lbm_destroy(lbm_handle *h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    drop_groups(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
}

}  // extern "C"
