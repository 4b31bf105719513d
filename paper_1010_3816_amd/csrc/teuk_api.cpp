// C ABI of libteuk.so (declared and documented in include/teuk.h).
//
// Host responsibilities: argument validation (before any device work),
// workspace layout, the 1-D coefficient tables of Eq. (1), extraction
// weights, launch geometry and ping-pong of the state buffers.  All step
// arithmetic runs in the gfx950 kernels of lw_kernels.hip.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/teuk.h"
#include "geometry.hpp"
#include "internal.hpp"

using namespace teuk;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(TEUK_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxExtract = 4096;
constexpr int kMaxFusedAdjointExtract = 16;  // extraction points handled inside the adjoint kernel
constexpr int64_t kMaxNr = int64_t(1) << 24;
constexpr int64_t kMaxNth = int64_t(1) << 20;
constexpr int kMinDefaultBlockSteps = 4;  // the default block pass takes at least this many steps a launch

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int pitch = 0;
    size_t state = 0;                 // bytes of one state [Phi, Pi][nth][pitch]
    size_t off_u[2]{};                // ping-pong state
    size_t off_rad = 0, off_ang = 0;  // KERR tables
    size_t off_uci = 0, off_uch = 0;  // USER tables
    size_t off_ext = 0, off_ext2 = 0, off_flag = 0;
    size_t total = 0;
};

int validate(const teuk_params* p) {
    if (!p) return fail(TEUK_E_INVALID_ARG, "params is NULL");
    if (!(p->a >= 0.0 && p->a < 1.0)) return fail(TEUK_E_INVALID_ARG, "spin a=%g outside [0, 1)", p->a);
    if (p->s < -2 || p->s > 2) return fail(TEUK_E_INVALID_ARG, "spin weight s=%d outside [-2, 2]", p->s);
    if (p->m < -1000 || p->m > 1000) return fail(TEUK_E_INVALID_ARG, "m=%d out of range", p->m);
    if (p->nr < 3 || p->nr > kMaxNr) return fail(TEUK_E_INVALID_ARG, "nr=%lld outside [3, 2^24]", (long long)p->nr);
    if (p->ntheta < 2 || p->ntheta > kMaxNth)
        return fail(TEUK_E_INVALID_ARG, "ntheta=%lld outside [2, 2^20]", (long long)p->ntheta);
    if (!std::isfinite(p->rstar_min) || !std::isfinite(p->rstar_max) || !(p->rstar_min < p->rstar_max))
        return fail(TEUK_E_INVALID_ARG, "need finite rstar_min < rstar_max");
    if (!std::isfinite(p->dt)) return fail(TEUK_E_INVALID_ARG, "dt=%g is not finite", p->dt);
    if (!(p->dt > 0.0) && p->coef_mode == TEUK_COEF_USER)
        return fail(TEUK_E_INVALID_ARG, "dt=%g: USER mode needs dt > 0", p->dt);
    if (p->coef_mode != TEUK_COEF_KERR && p->coef_mode != TEUK_COEF_USER)
        return fail(TEUK_E_INVALID_ARG, "coef_mode=%d unknown", p->coef_mode);
    if (p->n_extract < 0 || p->n_extract > kMaxExtract)
        return fail(TEUK_E_INVALID_ARG, "n_extract=%d outside [0, %d]", p->n_extract, kMaxExtract);
    if (p->n_extract > 0 && (!p->extract_rstar || !p->extract_theta))
        return fail(TEUK_E_INVALID_ARG, "extraction coordinates are NULL");
    const double nptr = (double)p->nr * (double)p->ntheta;
    if (nptr > 2.0e9) return fail(TEUK_E_INVALID_ARG, "nr*ntheta too large");
    for (int e = 0; e < p->n_extract; ++e) {
        const double r = p->extract_rstar[e], t = p->extract_theta[e];
        if (!(r >= p->rstar_min && r <= p->rstar_max))
            return fail(TEUK_E_INVALID_ARG, "extraction r*=%g outside the grid", r);
        if (!(t >= 0.0 && t <= M_PI)) return fail(TEUK_E_INVALID_ARG, "extraction theta=%g outside [0, pi]", t);
    }
    return TEUK_OK;
}

Layout make_layout(const teuk_params* p) {
    Layout L;
    const int nr = (int)p->nr, nth = (int)p->ntheta;
    L.pitch = (nr + 7) / 8 * 8;  // 128-byte rows of complex128
    L.state = align_up((size_t)nth * L.pitch * 2 * sizeof(double2));
    size_t o = 0;
    for (int k = 0; k < 2; ++k) {
        L.off_u[k] = o;
        o += L.state;
    }
    L.off_rad = o;
    o += align_up((size_t)kNumRad * 2 * L.pitch * sizeof(double));
    L.off_ang = o;
    o += align_up((size_t)kNumAng * nth * sizeof(double));
    if (p->coef_mode == TEUK_COEF_USER) {
        L.off_uci = o;
        o += align_up((size_t)kNumUser * nth * L.pitch * sizeof(double));
        L.off_uch = o;
        o += align_up((size_t)kNumUser * nth * L.pitch * sizeof(double));
    }
    L.off_ext = o;
    o += align_up(std::max(1, p->n_extract) * sizeof(ExtPoint));
    L.off_ext2 = o;
    o += align_up(kMaxExtract * sizeof(ExtPoint));
    L.off_flag = o;
    o += kAlign;
    L.total = o;
    return L;
}

// Bilinear weights of Phi at (r*, theta): columns col, col+1; rows rowa and
// rowb, with the pole ghost rows (sigma times the mirrored row) folded in.
ExtPoint ext_point(double rstar, double theta, double rmin, double dr, int nr, int nth, int sigma) {
    const double dth = M_PI / nth;
    const double pcol = (rstar - rmin) / dr;
    int col = (int)std::floor(pcol);
    col = std::min(std::max(col, 0), nr - 2);
    const double wr = pcol - col;
    const double qrow = theta / dth - 0.5;
    int j = (int)std::floor(qrow);
    j = std::min(std::max(j, -1), nth - 1);
    const double wt = qrow - j;
    ExtPoint E{};
    E.col = col;
    E.wr = wr;
    if (j < 0) {  // rows -1 (ghost of 0) and 0
        E.rowa = 0;
        E.wa = wt + sigma * (1.0 - wt);
        E.rowb = -1;
        E.wb = 0.0;
    } else if (j == nth - 1) {  // rows nth-1 and nth (ghost of nth-1)
        E.rowa = nth - 1;
        E.wa = (1.0 - wt) + sigma * wt;
        E.rowb = -1;
        E.wb = 0.0;
    } else {
        E.rowa = j;
        E.wa = 1.0 - wt;
        E.rowb = j + 1;
        E.wb = wt;
    }
    return E;
}

// Device scratch of teuk_extract_noalloc: the point records of one call,
// staged here instead of in a grid's workspace, so that the call needs no
// device memory from the caller beyond its output.  Every device the
// library runs on holds its own copy until the process ends.  Host code
// reaches a device's copy only through the address hipGetSymbolAddress
// returns for it with that device current (scratch_address), never through
// the array's name, which on the host is only a stand-in for the symbol.
constexpr int kNoAllocMaxPoints = kMaxExtract;
constexpr size_t kScratchBytes = (size_t)kNoAllocMaxPoints * sizeof(ExtPoint);  // 192 KiB
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;  // by device ordinal; nullptr until resolved

// Resolve the scratch address of `device`, which must be the current device
// (called once per device, from teuk_init_grid).
int resolve_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0) return fail(TEUK_E_HIP, "invalid device %d", device);
    if ((size_t)device < g_scratch_addr.size() && g_scratch_addr[device]) return TEUK_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(TEUK_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    if ((size_t)device >= g_scratch_addr.size()) g_scratch_addr.resize(device + 1, nullptr);
    g_scratch_addr[device] = p;
    return TEUK_OK;
}

void* scratch_address(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (device >= 0 && (size_t)device < g_scratch_addr.size()) ? g_scratch_addr[device] : nullptr;
}

}  // namespace

struct teuk_grid {
    teuk_params p{};
    std::vector<double> ext_r, ext_t;
    std::vector<ExtPoint> ext;
    Layout L;
    hipStream_t stream = nullptr;
    int device = 0;
    char* ws = nullptr;
    double dr = 0.0, dth = 0.0;
    int sigma = 1;
    int cur = 0;          // which ping-pong buffer holds the state
    int64_t steps = 0;
    int rows = 64;        // theta rows per wavefront tile
    int wpb = 4;          // wavefronts per workgroup
    bool fused_ext = true;
    int steps_per_pass = 2;  // 2: pairs of steps in one pass (temporal blocking)
    bool fused_ext2 = true;  // extraction fusable with the two-step strips
    int block_steps = 0;     // teuk_set_block_launch: steps per launch of the block pass (0: off)
    int block_cols = 0;      // columns a block-pass workgroup holds (0: not set)
    int64_t check_every = 0;  // teuk_set_finite_check: steps between device checks of the state (0: off)
    char* sws = nullptr;      // source profile (teuk_set_source): [integer, half][nth][pitch] complex128
    bool coef_set = false;
    // adjoint (teuk_enable_adjoint)
    char* aws = nullptr;      // adjoint workspace
    size_t aoff_lam[2]{}, aoff_da = 0, aoff_slots = 0, aoff_sum = 0;
    int adj_rows = 32, adj_wpb = 4, adj_chunks = 0, adj_strips = 0;  // spin-gradient and one-step kernels
    int adj2_rows = 32, adj2_chunks = 0;                              // two-step cotangent kernel
    int tan_rows = 32, tan_chunks = 0;                                // step-with-tangent kernel
    int cache_policy = TEUK_CACHE_AUTO;                               // teuk_set_cache_policy
    std::vector<double> x_tab;  // x = r - r_+ at the integer [0][nr] and half [1][nr] positions (KERR)
    // forward-mode spin derivative (teuk_enable_spin_tangent): v = du/da in two buffers
    char* tws = nullptr;
    int vcur = 0;

    double2* u(int k) const { return reinterpret_cast<double2*>(ws + L.off_u[k]); }
    double2* v(int k) const { return reinterpret_cast<double2*>(tws + (size_t)k * L.state); }
    template <class T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

// Fused extraction handles at most one point per tile (its state is held
// in scalar registers of the tile's wavefront).
bool fused_extraction_ok(const teuk_grid* g, int strip_cols = kStripCols, int rows = 0) {
    const auto& E = g->ext;
    if (rows <= 0) rows = g->rows;
    for (size_t i = 0; i < E.size(); ++i)
        for (size_t k = i + 1; k < E.size(); ++k)
            if (E[i].col / strip_cols == E[k].col / strip_cols && E[i].rowa / rows == E[k].rowa / rows)
                return false;
    return true;
}

void update_fusion(teuk_grid* g) {
    g->fused_ext = fused_extraction_ok(g);
    g->fused_ext2 = fused_extraction_ok(g, kStripCols2);
}

// Two states (a pass's input and output) up to this size stay in the
// last-level cache (256 MB on MI355X) with room to spare for the tables.
constexpr size_t kKeepStatesBytes = (size_t)192 << 20;

// Whether the next state is written with cache-keeping stores.
bool keeps_states(const teuk_grid* g) {
    if (g->cache_policy == TEUK_CACHE_KEEP) return true;
    if (g->cache_policy == TEUK_CACHE_STREAM) return false;
    return 2 * g->L.state <= kKeepStatesBytes;
}

StepArgs step_args(const teuk_grid* g) {
    StepArgs a{};
    StepScalars& k = a.k;
    k.nr = (int)g->p.nr;
    k.nth = (int)g->p.ntheta;
    k.pitch = g->L.pitch;
    k.sigma = g->sigma;
    k.rows = g->rows;
    k.n_strips = (k.nr + kStripCols - 1) / kStripCols;
    k.n_chunks = (k.nth + g->rows - 1) / g->rows;
    k.dt = g->p.dt;
    k.hdt = 0.5 * g->p.dt;
    k.dt_dr = g->p.dt / g->dr;
    k.hdt_dr = 0.5 * g->p.dt / g->dr;
    k.inv_dth2 = 1.0 / (g->dth * g->dth);
    k.inv_2dth = 1.0 / (2.0 * g->dth);
    k.plane = (int64_t)k.nth * k.pitch;
    a.rad = g->at<double>(g->L.off_rad);
    a.ang = g->at<double>(g->L.off_ang);
    if (g->p.coef_mode == TEUK_COEF_USER) {
        a.uci = g->at<double>(g->L.off_uci);
        a.uch = g->at<double>(g->L.off_uch);
    }
    a.ext = g->at<ExtPoint>(g->L.off_ext);
    k.n_ext = g->fused_ext ? g->p.n_extract : 0;
    k.keep = keeps_states(g) ? 1 : 0;
    return a;
}

int check_grid(const teuk_grid* g) {
    if (!g) return fail(TEUK_E_INVALID_ARG, "grid handle is NULL");
    return TEUK_OK;
}

// Bytes of one plane of the source profile ([nth][pitch] complex128).
size_t source_plane_bytes(const teuk_grid* g) { return align_up((size_t)g->p.ntheta * g->L.pitch * sizeof(double2)); }

// Status block of the workspace: [int] non-finite flag of teuk_check_finite,
// then at byte 8 the step count recorded by the first failing in-loop check
// (0: none).
long long* first_nonfinite(const teuk_grid* g) { return reinterpret_cast<long long*>(g->ws + g->L.off_flag + 8); }

// Default tile of the two-step pass.  The device holds two of its wavefronts
// per SIMD, so its tiles run in rounds of 8 x CUs; a last round that is only
// partly filled leaves SIMDs idle, and a wavefront walks its tile's rows one
// after the other, so on a grid that fits one round shorter tiles finish
// sooner.  Take the fewest rounds k whose tiles, cut so that the grid's tiles
// just fit k rounds, have at most 64 rows.  Grids with fewer tiles than SIMDs
// take one wavefront per workgroup, to spread over the CUs.
void default_tile(int nr, int nth, int cus, int* rows, int* wpb) {
    const int64_t strips2 = (nr + kStripCols2 - 1) / kStripCols2;
    const int64_t slots = (int64_t)cus * 8;
    int64_t r = 64;
    for (int64_t k = 1; k <= 64; ++k) {
        const int64_t chunks = k * slots / strips2;
        if (chunks < 1) continue;
        const int64_t rk = (nth + chunks - 1) / chunks;
        if (rk <= 64) {
            r = rk;
            break;
        }
    }
    r = std::min<int64_t>(r, nth);
    const int64_t tiles = strips2 * ((nth + r - 1) / r);
    *rows = (int)r;
    *wpb = tiles < (int64_t)cus * 4 ? 1 : 4;
}

// Default tile height of an adjoint kernel: the shortest tiles of which
// `slots` wavefronts hold all (workgroups take consecutive tiles of the
// strip-major list, so any tile count packs), at most 16 rows.
int adjoint_rows(int nr, int nth, int64_t slots, int strip_cols) {
    const int64_t strips = (nr + strip_cols - 1) / strip_cols;
    const int64_t chunks = slots / strips;  // theta chunks per strip
    if (chunks < 1) return std::min(nth, 16);
    return (int)std::min<int64_t>(std::min<int64_t>((nth + chunks - 1) / chunks, 16), nth);
}

int set_device(const teuk_grid* g) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != g->device) HIP_TRY(hipSetDevice(g->device));
    return TEUK_OK;
}

// Gershgorin bound of the largest |eigenvalue| of the discrete theta operator
// (rows of A2 (f+ - 2 f + f-)/dth^2 + A1 (f+ - f-)/(2 dth) - V0 f, ghost rows
// folded in) over all integer columns.
double angular_eig_bound(const teuk_params* p, double dr) {
    const int nr = (int)p->nr, nth = (int)p->ntheta;
    const double dth = M_PI / nth;
    const int sigma = (std::abs(p->m) % 2 == 0) ? 1 : -1;
    std::vector<double> ang((size_t)nth * kNumAng);
    for (int j = 0; j < nth; ++j) angular_fields(p->s, p->m, j, dth, &ang[(size_t)j * kNumAng]);
    double best = 0.0;
    for (int i = 0; i < nr; ++i) {
        double x;
        if (!tortoise_inverse(p->a, p->rstar_min + i * dr, &x)) continue;
        double R[kNumRad];
        radial_fields<double>(p->a, p->s, p->m, x, dth, R);
        for (int j = 0; j < nth; ++j) {
            const double* G = &ang[(size_t)j * kNumAng];
            const double inv = 1.0 / (R[R_RHO2] - R[R_A2D] * G[A_SN2]);
            const double a2 = R[R_DL2] * inv, a1 = a2 * G[A_COTP];
            const double v0 = std::hypot((R[R_DL2] * G[A_PD] + R[R_V0R]) * inv, R[R_V0I] * inv);
            double lo = a2 - a1, hi = a2 + a1, diag = -2.0 * a2;  // weights of f-, f+, f
            if (j == 0) diag += sigma * lo, lo = 0.0;
            if (j == nth - 1) diag += sigma * hi, hi = 0.0;
            best = std::max(best, std::fabs(diag) + v0 + std::fabs(lo) + std::fabs(hi));
        }
    }
    return best;
}

}  // namespace

extern "C" {

const char* teuk_last_error(void) { return g_last_error.c_str(); }

size_t teuk_workspace_bytes(const teuk_params* p) {
    if (validate(p) != TEUK_OK) return 0;
    return make_layout(p).total;
}

int teuk_radius(double a, double rstar, double* h_r) {
    if (!(a >= 0.0 && a < 1.0)) return fail(TEUK_E_INVALID_ARG, "spin a=%g outside [0, 1)", a);
    if (!std::isfinite(rstar) || !h_r) return fail(TEUK_E_INVALID_ARG, "need a finite r* and an output pointer");
    double x;
    if (!tortoise_inverse(a, rstar, &x)) return fail(TEUK_E_INVALID_ARG, "tortoise inversion failed at r*=%g", rstar);
    *h_r = 1.0 + std::sqrt(1.0 - a * a) + x;
    return TEUK_OK;
}

int teuk_suggest_dt(const teuk_params* p, int64_t n_steps, double growth, double courant, double* h_dt) {
    if (validate(p) != TEUK_OK) return TEUK_E_INVALID_ARG;
    if (!h_dt) return fail(TEUK_E_INVALID_ARG, "h_dt is NULL");
    if (n_steps < 1 || !(growth > 1.0) || !(courant > 0.0))
        return fail(TEUK_E_INVALID_ARG, "need n_steps >= 1, growth > 1, courant > 0");
    const double dr = (p->rstar_max - p->rstar_min) / (double)(p->nr - 1);
    const double w = std::sqrt(angular_eig_bound(p, dr));
    double dt = courant * dr;
    if (w > 0.0) dt = std::min(dt, std::pow(8.0 * std::log(growth) / (double)n_steps, 0.25) / w);
    *h_dt = dt;
    return TEUK_OK;
}

namespace {

// The grid's time step: the policy step for dt <= 0, the strict-mode check
// for dt > 0 with a horizon (see teuk_params in teuk.h).
constexpr int64_t kPolicySteps = 10000;
constexpr double kPolicyGrowth = 10.0;

int resolve_dt(const teuk_params* p, double* dt) {
    *dt = p->dt;
    if (p->coef_mode != TEUK_COEF_KERR) return TEUK_OK;
    const int64_t n = p->stable_steps > 0 ? p->stable_steps : kPolicySteps;
    if (!(p->dt > 0.0)) return teuk_suggest_dt(p, n, kPolicyGrowth, 0.5, dt);
    if (p->stable_steps > 0) {
        double bound = 0.0;
        if (int rc = teuk_suggest_dt(p, n, kPolicyGrowth, 1.0, &bound)) return rc;
        if (p->dt > bound)
            return fail(TEUK_E_UNSTABLE_DT,
                        "dt=%g exceeds %g: the fastest angular mode would grow more than %gx over %lld steps "
                        "(or the r* Courant number exceed 1)",
                        p->dt, bound, kPolicyGrowth, (long long)n);
    }
    return TEUK_OK;
}

}  // namespace

int teuk_init_grid(const teuk_params* p, void* hip_stream, void* d_workspace, size_t workspace_bytes,
                   teuk_grid** out) {
    if (int rc = validate(p)) return rc;
    double dt = 0.0;
    if (int rc = resolve_dt(p, &dt)) return rc;
    if (!out) return fail(TEUK_E_INVALID_ARG, "out is NULL");
    if (!d_workspace) return fail(TEUK_E_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
        return fail(TEUK_E_WORKSPACE, "workspace not %zu-byte aligned", kAlign);
    const Layout L = make_layout(p);
    if (workspace_bytes < L.total)
        return fail(TEUK_E_WORKSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, L.total);

    const int nr = (int)p->nr, nth = (int)p->ntheta;
    const double dr = (p->rstar_max - p->rstar_min) / (double)(nr - 1);
    const double dth = M_PI / nth;

    // 1-D tables on the host; x at each position is kept for the
    // a-derivative tables (teuk_enable_adjoint)
    std::vector<double> rad, ang((size_t)kNumAng * nth), xs;
    if (p->coef_mode == TEUK_COEF_KERR) {
        rad.assign((size_t)kNumRad * 2 * L.pitch, 0.0);
        xs.assign((size_t)2 * nr, 0.0);
        for (int kind = 0; kind < 2; ++kind) {
            const int npos = kind == 0 ? nr : nr - 1;
            for (int i = 0; i < npos; ++i) {
                const double rs = p->rstar_min + (i + 0.5 * kind) * dr;
                double x;
                if (!tortoise_inverse(p->a, rs, &x))
                    return fail(TEUK_E_INVALID_ARG, "tortoise inversion failed at r*=%g", rs);
                xs[(size_t)kind * nr + i] = x;
                double R[kNumRad];
                radial_fields<double>(p->a, p->s, p->m, x, dth, R);
                for (int f = 0; f < kNumRad; ++f) rad[((size_t)f * 2 + kind) * L.pitch + i] = R[f];
            }
        }
    }
    for (int j = 0; j < nth; ++j) {
        double G[kNumAng];
        angular_fields(p->s, p->m, j, dth, G);
        for (int f = 0; f < kNumAng; ++f) ang[(size_t)j * kNumAng + f] = G[f];
    }

    teuk_grid* g = new teuk_grid();
    g->p = *p;
    g->p.dt = dt;
    g->L = L;
    g->x_tab = std::move(xs);
    g->stream = reinterpret_cast<hipStream_t>(hip_stream);
    g->ws = reinterpret_cast<char*>(d_workspace);
    g->dr = dr;
    g->dth = dth;
    g->sigma = (std::abs(p->m) % 2 == 0) ? 1 : -1;
    int cus = 0;
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        default_tile(nr, nth, cus, &g->rows, &g->wpb);
    }
    // The block pass: one thread per point of (columns x all rows).  Default
    // launch: over workgroups of up to 256, 512 or 1024 threads (at most 64
    // columns), the most steps a launch (at least 4) whose workgroups fit the
    // device one per CU, scored by the per-step time measured on small grids
    // (400 x 16 .. 3200 x 32, 1600 x 64): about 0.8 ns per point a workgroup
    // holds plus 3.6 us per launch spread over its steps.
    if (nth <= kMaxBlockRows && g->p.coef_mode == TEUK_COEF_KERR) {
        double best = 0.0;
        for (int threads : {256, 512, 1024}) {
            const int c = std::min(64, threads / nth);
            if (c < 2 * kMinDefaultBlockSteps + 2) continue;
            for (int k = (c - 2) / 2; k >= kMinDefaultBlockSteps; --k) {
                const int64_t w = c - 2 * k;
                if ((nr + w - 1) / w > cus) continue;
                const double score = 0.8e-3 * c * nth + 3.6 / k;  // us per step
                if (g->block_steps == 0 || score < best) {
                    best = score;
                    g->block_steps = k;
                    g->block_cols = c;
                }
                break;  // the most steps for this width
            }
        }
    }
    // a device holds two adjoint wavefronts per SIMD (8 per CU).  The
    // spin-gradient kernel leaves one slot in eight to the recompute that
    // the reverse pass runs beside it; the two-step cotangent kernel, which
    // runs alone, fills the round.
    g->adj_rows = adjoint_rows(nr, nth, (int64_t)cus * 7, kStripCols);
    g->adj_chunks = (nth + g->adj_rows - 1) / g->adj_rows;
    g->adj2_rows = adjoint_rows(nr, nth, (int64_t)cus * 8, kStripCols2);
    g->adj2_chunks = (nth + g->adj2_rows - 1) / g->adj2_rows;
    g->tan_rows = adjoint_rows(nr, nth, (int64_t)cus * 8, kStripCols);
    g->tan_chunks = (nth + g->tan_rows - 1) / g->tan_rows;
    g->adj_strips = ((int)p->nr + kStripCols - 1) / kStripCols;
    g->ext_r.assign(p->extract_rstar, p->extract_rstar + p->n_extract);
    g->ext_t.assign(p->extract_theta, p->extract_theta + p->n_extract);
    g->p.extract_rstar = g->ext_r.data();
    g->p.extract_theta = g->ext_t.data();
    for (int e = 0; e < p->n_extract; ++e)
        g->ext.push_back(ext_point(g->ext_r[e], g->ext_t[e], p->rstar_min, dr, nr, nth, g->sigma));
    update_fusion(g);
    g->coef_set = p->coef_mode == TEUK_COEF_KERR;

    auto bail = [&](int rc) {
        delete g;
        return rc;
    };
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) return bail(fail(TEUK_E_HIP, "hipGetDevice: %s", hipGetErrorString(e)));
    if (int rc = resolve_scratch(g->device)) return bail(rc);
    hipStream_t s = g->stream;
    e = hipMemsetAsync(g->ws, 0, L.off_rad, s);  // both state buffers
    if (e == hipSuccess) e = hipMemsetAsync(g->ws + L.off_flag, 0, kAlign, s);  // status flags
    if (e == hipSuccess && !rad.empty())
        e = hipMemcpyAsync(g->ws + L.off_rad, rad.data(), rad.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->ws + L.off_ang, ang.data(), ang.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !g->ext.empty())
        e = hipMemcpyAsync(g->ws + L.off_ext, g->ext.data(), g->ext.size() * sizeof(ExtPoint),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(fail(TEUK_E_HIP, "uploading tables: %s", hipGetErrorString(e)));
    *out = g;
    return TEUK_OK;
}

int teuk_set_coefficients(teuk_grid* g, const double* d_ci, const double* d_ch) {
    if (int rc = check_grid(g)) return rc;
    if (g->p.coef_mode != TEUK_COEF_USER) return fail(TEUK_E_STATE, "grid is not in TEUK_COEF_USER mode");
    if (!d_ci || !d_ch) return fail(TEUK_E_INVALID_ARG, "coefficient pointers are NULL");
    if (int rc = set_device(g)) return rc;
    const int nr = (int)g->p.nr, nth = (int)g->p.ntheta;
    HIP_TRY(launch_pitch_copy(d_ci, g->at<double>(g->L.off_uci), kNumUser * nth, nr, g->L.pitch, g->stream));
    HIP_TRY(launch_pitch_copy(d_ch, g->at<double>(g->L.off_uch), kNumUser * nth, nr - 1, g->L.pitch, g->stream));
    g->coef_set = true;
    return TEUK_OK;
}

int teuk_set_initial_data(teuk_grid* g, const void* d_phi, const void* d_pi) {
    if (int rc = check_grid(g)) return rc;
    if (!d_phi || !d_pi) return fail(TEUK_E_INVALID_ARG, "initial data pointers are NULL");
    if (int rc = set_device(g)) return rc;
    const int nr = (int)g->p.nr, nth = (int)g->p.ntheta;
    HIP_TRY(launch_import(static_cast<const double2*>(d_phi), g->u(0), 0, nr, nth, g->L.pitch, g->stream));
    HIP_TRY(launch_import(static_cast<const double2*>(d_pi), g->u(0), 1, nr, nth, g->L.pitch, g->stream));
    g->cur = 0;
    g->steps = 0;
    return TEUK_OK;
}

namespace {

// Optional device check of the state every check_every steps (at the first
// pass boundary at or after each multiple) and at the end of a call: the
// first check that finds a non-finite value records its step count on the
// device; the call reads it once, at its end.
struct InLoopCheck {
    teuk_grid* g;
    long long* first_bad;
    int64_t start, last_check, next_check;
    explicit InLoopCheck(teuk_grid* grid)
        : g(grid), first_bad(first_nonfinite(grid)), start(grid->steps), last_check(grid->steps),
          next_check(grid->steps + grid->check_every) {}
    int check(const double2* u) {
        HIP_TRY(launch_nonfinite_step(u, (int)g->p.nr, (int)g->p.ntheta, g->L.pitch, first_bad, g->steps,
                                      g->stream));
        last_check = g->steps;
        return TEUK_OK;
    }
    int maybe(const double2* u) {
        if (g->check_every <= 0 || g->steps < next_check) return TEUK_OK;
        next_check = start + ((g->steps - start) / g->check_every + 1) * g->check_every;
        return check(u);
    }
    // u: the state after the call's last step
    int finish(const double2* u) {
        if (g->check_every <= 0) return TEUK_OK;
        if (last_check != g->steps)
            if (int rc = check(u)) return rc;
        long long bad = 0;
        HIP_TRY(hipMemcpyAsync(&bad, first_bad, sizeof(bad), hipMemcpyDeviceToHost, g->stream));
        HIP_TRY(hipStreamSynchronize(g->stream));
        if (bad) {
            HIP_TRY(launch_zero_ints(reinterpret_cast<int*>(first_bad), 2, g->stream));
            return fail(TEUK_E_NONFINITE, "the state holds a non-finite value, first seen by the check after step %lld",
                        bad);
        }
        return TEUK_OK;
    }
};

// n steps; optional extraction series and optional window of input states
// (slot k = the state before step k, stride L.state bytes); h_f: the time
// factors of the source term for the n steps (4 doubles per step), or
// nullptr for the homogeneous equation.
int step_n_impl(teuk_grid* g, int64_t n, void* d_series, void* d_window, const double* h_f = nullptr) {
    if (int rc = check_grid(g)) return rc;
    if (n < 0) return fail(TEUK_E_INVALID_ARG, "n=%lld < 0", (long long)n);
    if (!g->coef_set) return fail(TEUK_E_STATE, "USER-mode coefficients not set");
    if (n == 0) return TEUK_OK;
    if (int rc = set_device(g)) return rc;
    const int ne = g->p.n_extract;
    double2* series = (ne > 0) ? static_cast<double2*>(d_series) : nullptr;
    StepArgs a = step_args(g);
    if (h_f) {
        a.src_i = reinterpret_cast<const double2*>(g->sws);
        a.src_h = reinterpret_cast<const double2*>(g->sws + source_plane_bytes(g));
    }
    auto set_f = [&](StepScalars& k, int64_t step, int nsteps) {
        if (h_f)
            for (int j = 0; j < 4 * nsteps; ++j) k.sf[j] = h_f[4 * step + j];
    };
    const bool kerr = g->p.coef_mode == TEUK_COEF_KERR;
    const ExtPoint* ext = g->at<ExtPoint>(g->L.off_ext);
    char* win = static_cast<char*>(d_window);
    auto window_state = [&](int64_t k) { return reinterpret_cast<double2*>(win + (size_t)k * g->L.state); };
    // Without a window the state ping-pongs between the grid's two buffers.
    // With one, state k (0 < k < n) is written straight into window slot k,
    // the first step copies the grid's state into slot 0 on the way, and the
    // last step writes the grid's other buffer: no state is written twice.
    const int cur0 = g->cur;
    int cur = cur0;
    double2* in = g->u(cur0);
    auto next_buffer = [&](int64_t knext) -> double2* {
        if (win) return (knext < n) ? window_state(knext) : g->u(1 - cur0);
        return g->u(1 - cur);
    };
    auto advance = [&](double2* out) {
        if (!win) cur = 1 - cur;
        in = out;
    };
    // Pairs of steps run as one two-step pass (not the first step of a
    // window run, which also copies its input).
    const bool two = g->steps_per_pass == 2 && (ne == 0 || g->fused_ext2);
    StepArgs a2 = a;
    a2.k.n_strips = (a2.k.nr + kStripCols2 - 1) / kStripCols2;
    a2.k.n_ext = ne;
    // XCD runs of strips when each XCD gets at least 8 (measured: 0.6-0.8 %
    // faster on 25600 x 512 at 32-64 row tiles, neutral on 6400 x 256)
    a2.k.order = a2.k.n_strips >= 64 ? kTileOrderXcdStrip : kTileOrderDispatch;
    const int wpb2 = std::min(g->wpb, 4);
    // Sample of state j (after step j) goes to series row j-1.  Launches
    // with fused extraction sample their input (and a pass its intermediate
    // state); otherwise a separate pass samples each new state.
    const bool fused = g->fused_ext;
    int64_t sampled = 0;
    InLoopCheck chk(g);
    auto extract_state = [&](const double2* u, int64_t j) -> int {
        HIP_TRY(launch_extract(u, g->L.pitch, ext, ne, series + (j - 1) * ne, g->stream));
        sampled = j;
        return TEUK_OK;
    };
    // Small grids: launches of the block pass (not with a window, a source
    // term or a series of more extraction points than it samples).
    const bool block = g->block_steps > 0 && kerr && !win && !h_f && (!series || ne <= kMaxBlockExt);
    for (int64_t k = 0; k < n;) {
        if (block) {
            const int m = (int)std::min<int64_t>(g->block_steps, n - k);
            double2* out = next_buffer(k + m);
            StepArgs ab = a;
            ab.u_in = in;
            ab.u_out = out;
            ab.k.bsteps = m;
            ab.k.bcols = g->block_cols;
            ab.k.n_ext = series ? ne : 0;
            ab.k.row0 = k - 1;  // state k + s goes to series row k + s - 1
            ab.series = series;
            HIP_TRY(launch_block(ab, g->stream));
            if (series) sampled = k + m - 1;
            advance(out);
            k += m;
            g->steps += m;
            if (int rc = chk.maybe(in)) return rc;
            continue;
        }
        if (two && k + 2 <= n && !(win && k == 0)) {
            double2* out = next_buffer(k + 2);
            a2.u_in = in;
            a2.u_out = out;
            a2.win = win ? window_state(k + 1) : nullptr;
            a2.series = (series && k > 0) ? series + (k - 1) * ne : nullptr;
            a2.series_mid = series ? series + k * ne : nullptr;
            set_f(a2.k, k, 2);
            HIP_TRY(launch_step2(a2, kerr, wpb2, g->stream));
            if (series) sampled = k + 1;
            advance(out);
            k += 2;
            g->steps += 2;
            if (int rc = chk.maybe(in)) return rc;
        } else {
            if (series && !fused && k > sampled)
                if (int rc = extract_state(in, k)) return rc;
            double2* out = next_buffer(k + 1);
            a.u_in = in;
            a.u_out = out;
            a.win = (win && k == 0) ? window_state(0) : nullptr;
            a.series = (series && fused && k > 0) ? series + (k - 1) * ne : nullptr;
            set_f(a.k, k, 1);
            HIP_TRY(launch_step(a, kerr, g->wpb, g->stream));
            if (series && fused && k > 0) sampled = k;
            advance(out);
            k += 1;
            g->steps += 1;
            if (series && !fused)
                if (int rc = extract_state(out, k)) return rc;
            if (int rc = chk.maybe(in)) return rc;
        }
    }
    if (series && sampled < n)
        if (int rc = extract_state(in, n)) return rc;
    g->cur = win ? 1 - cur0 : cur;
    return chk.finish(in);
}

}  // namespace

int teuk_step_n(teuk_grid* g, int64_t n, void* d_series) { return step_n_impl(g, n, d_series, nullptr); }

size_t teuk_source_workspace_bytes(const teuk_grid* g) {
    if (!g) {
        fail(TEUK_E_INVALID_ARG, "grid handle is NULL");
        return 0;
    }
    return 2 * source_plane_bytes(g);
}

int teuk_set_source(teuk_grid* g, void* d_src_workspace, size_t bytes, const void* d_gi, const void* d_gh) {
    if (int rc = check_grid(g)) return rc;
    if (!d_gi && !d_gh) {
        g->sws = nullptr;
        return TEUK_OK;
    }
    if (!d_gi || !d_gh) return fail(TEUK_E_INVALID_ARG, "give both source profiles or neither");
    if (!d_src_workspace) return fail(TEUK_E_INVALID_ARG, "source workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_src_workspace) % kAlign)
        return fail(TEUK_E_WORKSPACE, "source workspace not %zu-byte aligned", kAlign);
    if (bytes < 2 * source_plane_bytes(g))
        return fail(TEUK_E_WORKSPACE, "source workspace has %zu bytes, needs %zu", bytes, 2 * source_plane_bytes(g));
    if (int rc = set_device(g)) return rc;
    const int nr = (int)g->p.nr, nth = (int)g->p.ntheta, P = g->L.pitch;
    char* ws = static_cast<char*>(d_src_workspace);
    // complex128 rows as pairs of doubles: dense [nth][cols] -> pitched [nth][pitch]
    HIP_TRY(launch_pitch_copy(static_cast<const double*>(d_gi), reinterpret_cast<double*>(ws), nth, 2 * nr, 2 * P,
                              g->stream));
    HIP_TRY(launch_pitch_copy(static_cast<const double*>(d_gh), reinterpret_cast<double*>(ws + source_plane_bytes(g)),
                              nth, 2 * (nr - 1), 2 * P, g->stream));
    g->sws = ws;
    return TEUK_OK;
}

int teuk_step_n_source(teuk_grid* g, int64_t n, void* d_series, const double* h_f) {
    if (int rc = check_grid(g)) return rc;
    if (!g->sws) return fail(TEUK_E_STATE, "no source profile: call teuk_set_source first");
    if (n > 0 && !h_f) return fail(TEUK_E_INVALID_ARG, "time factors are NULL");
    for (int64_t j = 0; j < 4 * n; ++j)
        if (!std::isfinite(h_f[j])) return fail(TEUK_E_INVALID_ARG, "time factor %lld is not finite", (long long)j);
    return step_n_impl(g, n, d_series, nullptr, h_f);
}

size_t teuk_window_bytes(const teuk_grid* g, int64_t n) {
    if (!g || n < 0) {
        fail(TEUK_E_INVALID_ARG, "need a grid and n >= 0");
        return 0;
    }
    return g->L.state * (size_t)n;
}

int teuk_step_n_store(teuk_grid* g, int64_t n, void* d_series, void* d_window) {
    if (n > 0 && !d_window) return fail(TEUK_E_INVALID_ARG, "window is NULL");
    if (d_window && reinterpret_cast<uintptr_t>(d_window) % kAlign)
        return fail(TEUK_E_WORKSPACE, "window not %zu-byte aligned", kAlign);
    return step_n_impl(g, n, d_series, d_window);
}

namespace {

// Host check of the extraction requests of teuk_extract / teuk_extract_noalloc.
int check_extract_args(const teuk_grid* g, int32_t n, int32_t max_n, const double* h_rstar, const double* h_theta,
                       const void* d_out) {
    if (int rc = check_grid(g)) return rc;
    if (n < 0 || n > max_n) return fail(TEUK_E_INVALID_ARG, "n=%d outside [0, %d]", n, max_n);
    if (n == 0) return TEUK_OK;
    if (!h_rstar || !h_theta || !d_out) return fail(TEUK_E_INVALID_ARG, "NULL pointer");
    for (int e = 0; e < n; ++e) {
        if (!(h_rstar[e] >= g->p.rstar_min && h_rstar[e] <= g->p.rstar_max))
            return fail(TEUK_E_INVALID_ARG, "r*=%g outside the grid", h_rstar[e]);
        if (!(h_theta[e] >= 0.0 && h_theta[e] <= M_PI))
            return fail(TEUK_E_INVALID_ARG, "theta=%g outside [0, pi]", h_theta[e]);
    }
    return TEUK_OK;
}

ExtPoint grid_ext_point(const teuk_grid* g, double rstar, double theta) {
    return ext_point(rstar, theta, g->p.rstar_min, g->dr, (int)g->p.nr, (int)g->p.ntheta, g->sigma);
}

}  // namespace

int teuk_get_window_slot(teuk_grid* g, const void* d_window, int64_t k, void* d_phi, void* d_pi) {
    if (int rc = check_grid(g)) return rc;
    if (!d_window || !d_phi || !d_pi) return fail(TEUK_E_INVALID_ARG, "NULL pointer");
    if (k < 0) return fail(TEUK_E_INVALID_ARG, "slot %lld < 0", (long long)k);
    if (int rc = set_device(g)) return rc;
    const int nr = (int)g->p.nr, nth = (int)g->p.ntheta;
    const double2* u = reinterpret_cast<const double2*>(static_cast<const char*>(d_window) + (size_t)k * g->L.state);
    HIP_TRY(launch_export(u, static_cast<double2*>(d_phi), 0, nr, nth, g->L.pitch, g->stream));
    HIP_TRY(launch_export(u, static_cast<double2*>(d_pi), 1, nr, nth, g->L.pitch, g->stream));
    return TEUK_OK;
}

int teuk_extract(teuk_grid* g, int32_t n, const double* h_rstar, const double* h_theta, void* d_out) {
    if (int rc = check_extract_args(g, n, kMaxExtract, h_rstar, h_theta, d_out)) return rc;
    if (n == 0) return TEUK_OK;
    std::vector<ExtPoint> pts(n);
    for (int e = 0; e < n; ++e) pts[e] = grid_ext_point(g, h_rstar[e], h_theta[e]);
    if (int rc = set_device(g)) return rc;
    ExtPoint* dp = g->at<ExtPoint>(g->L.off_ext2);
    HIP_TRY(hipMemcpyAsync(dp, pts.data(), n * sizeof(ExtPoint), hipMemcpyHostToDevice, g->stream));
    HIP_TRY(launch_extract(g->u(g->cur), g->L.pitch, dp, n, static_cast<double2*>(d_out), g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));  // `pts` is released on return
    return TEUK_OK;
}

int teuk_extract_noalloc(teuk_grid* g, int32_t n, const double* h_rstar, const double* h_theta, void* d_out) {
    if (int rc = check_extract_args(g, n, kNoAllocMaxPoints, h_rstar, h_theta, d_out)) return rc;
    if (n == 0) return TEUK_OK;
    if (int rc = set_device(g)) return rc;
    char* d_scratch = static_cast<char*>(scratch_address(g->device));
    if (!d_scratch) return fail(TEUK_E_STATE, "no scratch address for device %d", g->device);
    // The point records are built in stack chunks and staged into this
    // device's scratch; a chunk buffer is reused only once its copy is done.
    constexpr int kChunk = 256;
    ExtPoint buf[kChunk];
    for (int e0 = 0; e0 < n; e0 += kChunk) {
        const int c = std::min(kChunk, n - e0);
        for (int k = 0; k < c; ++k) buf[k] = grid_ext_point(g, h_rstar[e0 + k], h_theta[e0 + k]);
        HIP_TRY(hipMemcpyAsync(d_scratch + (size_t)e0 * sizeof(ExtPoint), buf, c * sizeof(ExtPoint),
                               hipMemcpyHostToDevice, g->stream));
        HIP_TRY(hipStreamSynchronize(g->stream));
    }
    HIP_TRY(launch_extract(g->u(g->cur), g->L.pitch, reinterpret_cast<const ExtPoint*>(d_scratch), n,
                           static_cast<double2*>(d_out), g->stream));
    // the scratch is free for the next call once this one returns
    HIP_TRY(hipStreamSynchronize(g->stream));
    return TEUK_OK;
}

int teuk_get_state(teuk_grid* g, void* d_phi, void* d_pi) {
    if (int rc = check_grid(g)) return rc;
    if (!d_phi || !d_pi) return fail(TEUK_E_INVALID_ARG, "output pointers are NULL");
    if (int rc = set_device(g)) return rc;
    const int nr = (int)g->p.nr, nth = (int)g->p.ntheta;
    HIP_TRY(launch_export(g->u(g->cur), static_cast<double2*>(d_phi), 0, nr, nth, g->L.pitch, g->stream));
    HIP_TRY(launch_export(g->u(g->cur), static_cast<double2*>(d_pi), 1, nr, nth, g->L.pitch, g->stream));
    return TEUK_OK;
}

int teuk_check_finite(teuk_grid* g) {
    if (int rc = check_grid(g)) return rc;
    if (int rc = set_device(g)) return rc;
    int* flag = g->at<int>(g->L.off_flag);
    HIP_TRY(launch_zero_ints(flag, 1, g->stream));
    HIP_TRY(launch_nonfinite(g->u(g->cur), (int)g->p.nr, (int)g->p.ntheta, g->L.pitch, flag, g->stream));
    int h = 0;
    HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    if (h) return fail(TEUK_E_NONFINITE, "state holds a non-finite value after %lld steps", (long long)g->steps);
    return TEUK_OK;
}

int teuk_set_finite_check(teuk_grid* g, int64_t every) {
    if (int rc = check_grid(g)) return rc;
    if (every < 0) return fail(TEUK_E_INVALID_ARG, "every=%lld < 0", (long long)every);
    g->check_every = every;
    return TEUK_OK;
}

int64_t teuk_steps_taken(const teuk_grid* g) { return g ? g->steps : -1; }

double teuk_get_dt(const teuk_grid* g) { return g ? g->p.dt : 0.0; }

int teuk_set_tile(teuk_grid* g, int32_t rows_per_tile, int32_t waves_per_block) {
    if (int rc = check_grid(g)) return rc;
    if (rows_per_tile < 1 || rows_per_tile > g->p.ntheta)
        return fail(TEUK_E_INVALID_ARG, "rows_per_tile=%d outside [1, ntheta]", rows_per_tile);
    if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4 && waves_per_block != 8)
        return fail(TEUK_E_INVALID_ARG, "waves_per_block=%d not in {1, 2, 4, 8}", waves_per_block);
    g->rows = rows_per_tile;
    g->wpb = waves_per_block;
    update_fusion(g);
    return TEUK_OK;
}

int teuk_set_steps_per_pass(teuk_grid* g, int32_t steps_per_pass) {
    if (int rc = check_grid(g)) return rc;
    if (steps_per_pass != 1 && steps_per_pass != 2)
        return fail(TEUK_E_INVALID_ARG, "steps_per_pass=%d not in {1, 2}", steps_per_pass);
    g->steps_per_pass = steps_per_pass;
    return TEUK_OK;
}

int teuk_get_steps_per_pass(const teuk_grid* g, int32_t* steps_per_pass) {
    if (int rc = check_grid(g)) return rc;
    if (steps_per_pass) *steps_per_pass = g->steps_per_pass;
    return TEUK_OK;
}

int teuk_set_block_launch(teuk_grid* g, int32_t steps, int32_t cols) {
    if (int rc = check_grid(g)) return rc;
    if (steps == 0) {
        g->block_steps = 0;
        return TEUK_OK;
    }
    const int nth = (int)g->p.ntheta;
    if (g->p.coef_mode != TEUK_COEF_KERR || nth > kMaxBlockRows)
        return fail(TEUK_E_INVALID_ARG, "the block pass needs Kerr coefficients and ntheta <= %d", kMaxBlockRows);
    if (cols == 0) cols = g->block_cols > 0 ? g->block_cols : std::min(64, 1024 / nth);
    if (cols < 4 || cols > 64 || cols * nth > 1024)
        return fail(TEUK_E_INVALID_ARG, "block cols=%d outside [4, min(64, 1024/ntheta=%d)]", cols, 1024 / nth);
    if (steps < 0 || steps > (cols - 2) / 2)
        return fail(TEUK_E_INVALID_ARG, "block steps=%d outside [0, %d] for %d columns", steps, (cols - 2) / 2, cols);
    g->block_steps = steps;
    g->block_cols = cols;
    return TEUK_OK;
}

int teuk_get_block_launch(const teuk_grid* g, int32_t* steps, int32_t* cols) {
    if (int rc = check_grid(g)) return rc;
    if (steps) *steps = g->block_steps;
    if (cols) *cols = g->block_cols;
    return TEUK_OK;
}

int teuk_set_cache_policy(teuk_grid* g, int32_t policy) {
    if (int rc = check_grid(g)) return rc;
    if (policy != TEUK_CACHE_AUTO && policy != TEUK_CACHE_KEEP && policy != TEUK_CACHE_STREAM)
        return fail(TEUK_E_INVALID_ARG, "cache policy %d not in {0, 1, 2}", policy);
    g->cache_policy = policy;
    return TEUK_OK;
}

int teuk_get_cache_policy(const teuk_grid* g, int32_t* policy, int32_t* keeps) {
    if (int rc = check_grid(g)) return rc;
    if (policy) *policy = g->cache_policy;
    if (keeps) *keeps = keeps_states(g) ? 1 : 0;
    return TEUK_OK;
}

int teuk_get_tile(const teuk_grid* g, int32_t* rows_per_tile, int32_t* waves_per_block) {
    if (int rc = check_grid(g)) return rc;
    if (rows_per_tile) *rows_per_tile = g->rows;
    if (waves_per_block) *waves_per_block = g->wpb;
    return TEUK_OK;
}

int teuk_set_adjoint_tile(teuk_grid* g, int32_t rows_per_tile, int32_t waves_per_block) {
    if (int rc = check_grid(g)) return rc;
    if (rows_per_tile < 1 || rows_per_tile > g->p.ntheta)
        return fail(TEUK_E_INVALID_ARG, "rows_per_tile=%d outside [1, ntheta]", rows_per_tile);
    if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
        return fail(TEUK_E_INVALID_ARG, "waves_per_block=%d not in {1, 2, 4}", waves_per_block);
    g->adj_rows = g->adj2_rows = g->tan_rows = rows_per_tile;
    g->adj_chunks = g->adj2_chunks = g->tan_chunks = (int)((g->p.ntheta + rows_per_tile - 1) / rows_per_tile);
    g->adj_wpb = waves_per_block;
    return TEUK_OK;
}

int teuk_get_adjoint_tile(const teuk_grid* g, int32_t* rows_per_tile, int32_t* waves_per_block) {
    if (int rc = check_grid(g)) return rc;
    if (rows_per_tile) *rows_per_tile = g->adj_rows;
    if (waves_per_block) *waves_per_block = g->adj_wpb;
    return TEUK_OK;
}

namespace {

void adjoint_layout(teuk_grid* g, size_t* total) {
    const int nth = (int)g->p.ntheta;
    size_t o = 0;
    for (int k = 0; k < 2; ++k) {
        g->aoff_lam[k] = o;
        o += g->L.state;
    }
    g->aoff_da = o;
    o += align_up((size_t)kNumRad * 2 * g->L.pitch * sizeof(double));
    g->aoff_slots = o;
    // one slot per tile of either adjoint tiling, for any tile rows
    const size_t strips2 = ((size_t)g->p.nr + kStripCols2 - 1) / kStripCols2;
    o += align_up(std::max<size_t>(g->adj_strips, strips2) * nth * sizeof(double));
    g->aoff_sum = o;
    o += kAlign;
    *total = o;
}

}  // namespace

size_t teuk_adjoint_workspace_bytes(teuk_grid* g) {
    if (!g) {
        fail(TEUK_E_INVALID_ARG, "grid handle is NULL");
        return 0;
    }
    size_t total;
    adjoint_layout(g, &total);
    return total;
}

int teuk_enable_adjoint(teuk_grid* g, void* d_adj_workspace, size_t bytes) {
    if (int rc = check_grid(g)) return rc;
    if (g->p.coef_mode != TEUK_COEF_KERR) return fail(TEUK_E_STATE, "the adjoint needs TEUK_COEF_KERR coefficients");
    if (!d_adj_workspace) return fail(TEUK_E_INVALID_ARG, "adjoint workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_adj_workspace) % kAlign)
        return fail(TEUK_E_WORKSPACE, "adjoint workspace not %zu-byte aligned", kAlign);
    size_t total;
    adjoint_layout(g, &total);
    if (bytes < total) return fail(TEUK_E_WORKSPACE, "adjoint workspace has %zu bytes, needs %zu", bytes, total);
    // a-derivatives of the radial tables at fixed r* (dual numbers through
    // the tortoise inversion and every radial factor), from the x that
    // teuk_init_grid solved for at each position
    const int nr = (int)g->p.nr;
    std::vector<double> da((size_t)kNumRad * 2 * g->L.pitch, 0.0);
    for (int kind = 0; kind < 2; ++kind) {
        const int npos = kind == 0 ? nr : nr - 1;
        for (int i = 0; i < npos; ++i) {
            const Dual x = tortoise_x_dual(g->p.a, g->x_tab[(size_t)kind * nr + i]);
            Dual R[kNumRad];
            radial_fields<Dual>(Dual(g->p.a, 1.0), g->p.s, g->p.m, x, g->dth, R);
            for (int f = 0; f < kNumRad; ++f) da[((size_t)f * 2 + kind) * g->L.pitch + i] = R[f].d;
        }
    }
    if (int rc = set_device(g)) return rc;
    g->aws = static_cast<char*>(d_adj_workspace);
    HIP_TRY(hipMemsetAsync(g->aws, 0, total, g->stream));
    HIP_TRY(hipMemcpyAsync(g->aws + g->aoff_da, da.data(), da.size() * sizeof(double), hipMemcpyHostToDevice,
                           g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    return TEUK_OK;
}

namespace {

// Launch arguments of the adjoint-side kernels (tiles of the one-step
// adjoint kernel; callers adjust rows, strips and chunks for the others).
AdjArgs adjoint_args(const teuk_grid* g) {
    AdjArgs a{};
    const int nth = (int)g->p.ntheta;
    a.k.nr = (int)g->p.nr;
    a.k.nth = nth;
    a.k.pitch = g->L.pitch;
    a.k.sigma = g->sigma;
    a.k.rows = g->adj_rows;
    a.k.n_strips = g->adj_strips;
    a.k.n_chunks = g->adj_chunks;
    a.k.zero = 0;
    a.k.keep = keeps_states(g) ? 1 : 0;
    a.k.plane = (int64_t)nth * g->L.pitch;
    a.k.dt = g->p.dt;
    a.k.hdt = 0.5 * g->p.dt;
    a.k.dt_dr = g->p.dt / g->dr;
    a.k.hdt_dr = 0.5 * g->p.dt / g->dr;
    a.rad = g->at<double>(g->L.off_rad);
    a.rad_da = reinterpret_cast<const double*>(g->aws + g->aoff_da);
    a.ang = g->at<double>(g->L.off_ang);
    a.ext = g->at<ExtPoint>(g->L.off_ext);
    return a;
}

}  // namespace

int teuk_step_n_tangent(teuk_grid* g, int64_t n, void* d_window) {
    if (int rc = check_grid(g)) return rc;
    if (n < 0) return fail(TEUK_E_INVALID_ARG, "n=%lld < 0", (long long)n);
    if (!g->aws) return fail(TEUK_E_STATE, "teuk_enable_adjoint has not been called");
    if (n > 0 && !d_window) return fail(TEUK_E_INVALID_ARG, "window is NULL");
    if (d_window && reinterpret_cast<uintptr_t>(d_window) % kAlign)
        return fail(TEUK_E_WORKSPACE, "window not %zu-byte aligned", kAlign);
    if (n == 0) return TEUK_OK;
    if (int rc = set_device(g)) return rc;
    AdjArgs a = adjoint_args(g);
    a.k.rows = g->tan_rows;
    a.k.n_chunks = g->tan_chunks;
    char* win = static_cast<char*>(d_window);
    for (int64_t k = 0; k < n; ++k) {
        double2* t_out = reinterpret_cast<double2*>(win + (size_t)k * g->L.state);
        HIP_TRY(launch_tangent(g->u(g->cur), g->u(1 - g->cur), t_out, a, g->adj_wpb, g->stream));
        g->cur = 1 - g->cur;
        g->steps += 1;
    }
    return TEUK_OK;
}

namespace {

// The reverse of a segment; dL/da goes to the host (h_acc: reduced,
// copied back, synchronised) or to a device accumulator (d_acc: added on the
// stream, asynchronous), or nowhere (both NULL: cotangents only).
int adjoint_impl(teuk_grid* g, int64_t n, void* d_lam_phi, void* d_lam_pi, const void* d_dL_dseries,
                 const void* d_window, int32_t flags, double* h_dL_da_accum, double* d_dL_da_accum) {
    if (int rc = check_grid(g)) return rc;
    if (!g->aws) return fail(TEUK_E_STATE, "teuk_enable_adjoint has not been called");
    if (n < 0) return fail(TEUK_E_INVALID_ARG, "n=%lld < 0", (long long)n);
    if (!d_lam_phi || !d_lam_pi) return fail(TEUK_E_INVALID_ARG, "cotangent pointers are NULL");
    // without a dL/da accumulator only the cotangents are computed, and they
    // do not depend on the forward states (the step is linear)
    const bool spin = h_dL_da_accum != nullptr || d_dL_da_accum != nullptr;
    if (n > 0 && spin && !d_window) return fail(TEUK_E_INVALID_ARG, "window is NULL");
    if (flags & ~(TEUK_ADJ_PROJECT_INITIAL | TEUK_ADJ_TANGENT_WINDOW))
        return fail(TEUK_E_INVALID_ARG, "unknown flags 0x%x", flags);
    // the window holds T_k = (dA/da) u^k (teuk_step_n_tangent) instead of u^k
    const bool tangent = spin && (flags & TEUK_ADJ_TANGENT_WINDOW);
    if (int rc = set_device(g)) return rc;
    const int nr = (int)g->p.nr, nth = (int)g->p.ntheta, P = g->L.pitch;
    const int ne = g->p.n_extract;
    const double2* gs = (ne > 0) ? static_cast<const double2*>(d_dL_dseries) : nullptr;
    const ExtPoint* ext = g->at<ExtPoint>(g->L.off_ext);
    hipStream_t s = g->stream;
    auto lam = [&](int k) { return reinterpret_cast<double2*>(g->aws + g->aoff_lam[k]); };
    double* slots = reinterpret_cast<double*>(g->aws + g->aoff_slots);
    double* sum = reinterpret_cast<double*>(g->aws + g->aoff_sum);
    const int strips2 = (nr + kStripCols2 - 1) / kStripCols2;
    const int nslots = std::max(g->adj_strips * g->adj_chunks, strips2 * g->adj2_chunks);

    int c = 0;
    HIP_TRY(launch_import(static_cast<const double2*>(d_lam_phi), lam(c), 0, nr, nth, P, s));
    HIP_TRY(launch_import(static_cast<const double2*>(d_lam_pi), lam(c), 1, nr, nth, P, s));
    if (spin) {
        HIP_TRY(hipMemsetAsync(slots, 0, (size_t)nslots * sizeof(double), s));
        if (!d_dL_da_accum) HIP_TRY(hipMemsetAsync(sum, 0, sizeof(double), s));
    }
    // the sample of the segment's last state
    if (gs && n > 0) HIP_TRY(launch_extract_adjoint(lam(c), P, ext, ne, gs + (n - 1) * ne, s));
    AdjArgs a = adjoint_args(g);
    a.slots = slots;
    // the sample of the state an adjoint step produces is added by the
    // adjoint kernel itself for a few points, by a separate pass otherwise
    const bool fused = ne <= kMaxFusedAdjointExtract;
    a.k.n_ext = fused ? ne : 0;
    const char* win = static_cast<const char*>(d_window);
    auto slot = [&](int64_t k) { return reinterpret_cast<const double2*>(win + (size_t)k * g->L.state); };
    int64_t k = n - 1;
    if ((!spin || tangent) && fused && g->steps_per_pass == 2) {
        // cotangents (and the tangents' dot products): two adjoint steps
        // (k, then k-1) per pass
        AdjArgs a2 = a;
        a2.k.n_strips = strips2;
        a2.k.rows = g->adj2_rows;
        a2.k.n_chunks = g->adj2_chunks;
        for (; k >= 1; k -= 2) {
            a2.nu_in = lam(c);
            a2.lam_out = lam(1 - c);
            a2.u_in = tangent ? slot(k) : nullptr;
            a2.gsample = gs ? reinterpret_cast<const double*>(gs + (k - 1) * ne) : nullptr;
            const double* gb = (gs && k >= 2) ? reinterpret_cast<const double*>(gs + (k - 2) * ne) : nullptr;
            HIP_TRY(launch_adjoint2(a2, gb, tangent ? slot(k - 1) : nullptr, g->adj_wpb, s));
            c = 1 - c;
        }
    }
    const AdjMode mode = tangent ? AdjMode::kTangentDot : spin ? AdjMode::kSpin : AdjMode::kCotangent;
    for (; k >= 0; --k) {
        a.nu_in = lam(c);
        a.u_in = spin ? slot(k) : nullptr;
        a.lam_out = lam(1 - c);
        a.gsample = (gs && k >= 1 && fused) ? reinterpret_cast<const double*>(gs + (k - 1) * ne) : nullptr;
        HIP_TRY(launch_adjoint(a, g->adj_wpb, mode, s));
        c = 1 - c;
        if (gs && k >= 1 && !fused) HIP_TRY(launch_extract_adjoint(lam(c), P, ext, ne, gs + (k - 1) * ne, s));
    }
    if (flags & TEUK_ADJ_PROJECT_INITIAL) HIP_TRY(launch_zero_radial_boundary(lam(c), nr, nth, P, s));
    HIP_TRY(launch_export(lam(c), static_cast<double2*>(d_lam_phi), 0, nr, nth, P, s));
    HIP_TRY(launch_export(lam(c), static_cast<double2*>(d_lam_pi), 1, nr, nth, P, s));
    if (!spin) return TEUK_OK;  // asynchronous
    if (d_dL_da_accum) {         // asynchronous: added on the stream, in call order
        HIP_TRY(launch_reduce_slots(slots, nslots, d_dL_da_accum, s));
        return TEUK_OK;
    }
    HIP_TRY(launch_reduce_slots(slots, nslots, sum, s));
    double h = 0.0;
    HIP_TRY(hipMemcpyAsync(&h, sum, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *h_dL_da_accum += h;
    return TEUK_OK;
}

}  // namespace

int teuk_adjoint_step_n(teuk_grid* g, int64_t n, void* d_lam_phi, void* d_lam_pi, const void* d_dL_dseries,
                        const void* d_window, int32_t flags, double* h_dL_da_accum) {
    return adjoint_impl(g, n, d_lam_phi, d_lam_pi, d_dL_dseries, d_window, flags, h_dL_da_accum, nullptr);
}

int teuk_adjoint_step_n_async(teuk_grid* g, int64_t n, void* d_lam_phi, void* d_lam_pi, const void* d_dL_dseries,
                              const void* d_window, int32_t flags, double* d_dL_da_accum) {
    if (!d_dL_da_accum) return fail(TEUK_E_INVALID_ARG, "the dL/da accumulator is NULL");
    return adjoint_impl(g, n, d_lam_phi, d_lam_pi, d_dL_dseries, d_window, flags, nullptr, d_dL_da_accum);
}

/* ---- forward-mode spin derivative ------------------------------------- */

size_t teuk_spin_tangent_workspace_bytes(const teuk_grid* g) {
    if (!g) {
        fail(TEUK_E_INVALID_ARG, "grid handle is NULL");
        return 0;
    }
    return 2 * g->L.state;
}

int teuk_enable_spin_tangent(teuk_grid* g, void* d_workspace, size_t bytes) {
    if (int rc = check_grid(g)) return rc;
    if (!g->aws) return fail(TEUK_E_STATE, "teuk_enable_adjoint has not been called (it builds the a-derivative tables)");
    if (!d_workspace) return fail(TEUK_E_INVALID_ARG, "spin-tangent workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
        return fail(TEUK_E_WORKSPACE, "spin-tangent workspace not %zu-byte aligned", kAlign);
    if (bytes < 2 * g->L.state)
        return fail(TEUK_E_WORKSPACE, "spin-tangent workspace has %zu bytes, needs %zu", bytes, 2 * g->L.state);
    if (int rc = set_device(g)) return rc;
    g->tws = static_cast<char*>(d_workspace);
    g->vcur = 0;
    HIP_TRY(hipMemsetAsync(g->tws, 0, 2 * g->L.state, g->stream));
    return TEUK_OK;
}

int teuk_set_spin_tangent(teuk_grid* g, const void* d_vphi, const void* d_vpi) {
    if (int rc = check_grid(g)) return rc;
    if (!g->tws) return fail(TEUK_E_STATE, "teuk_enable_spin_tangent has not been called");
    if ((d_vphi == nullptr) != (d_vpi == nullptr)) return fail(TEUK_E_INVALID_ARG, "give both planes or neither");
    if (int rc = set_device(g)) return rc;
    g->vcur = 0;
    if (!d_vphi) {
        HIP_TRY(hipMemsetAsync(g->v(0), 0, g->L.state, g->stream));
        return TEUK_OK;
    }
    const int nr = (int)g->p.nr, nth = (int)g->p.ntheta;
    HIP_TRY(launch_import(static_cast<const double2*>(d_vphi), g->v(0), 0, nr, nth, g->L.pitch, g->stream));
    HIP_TRY(launch_import(static_cast<const double2*>(d_vpi), g->v(0), 1, nr, nth, g->L.pitch, g->stream));
    return TEUK_OK;
}

int teuk_get_spin_tangent(teuk_grid* g, void* d_vphi, void* d_vpi) {
    if (int rc = check_grid(g)) return rc;
    if (!g->tws) return fail(TEUK_E_STATE, "teuk_enable_spin_tangent has not been called");
    if (!d_vphi || !d_vpi) return fail(TEUK_E_INVALID_ARG, "output pointers are NULL");
    if (int rc = set_device(g)) return rc;
    const int nr = (int)g->p.nr, nth = (int)g->p.ntheta;
    HIP_TRY(launch_export(g->v(g->vcur), static_cast<double2*>(d_vphi), 0, nr, nth, g->L.pitch, g->stream));
    HIP_TRY(launch_export(g->v(g->vcur), static_cast<double2*>(d_vpi), 1, nr, nth, g->L.pitch, g->stream));
    return TEUK_OK;
}

int teuk_step_n_spin_tangent(teuk_grid* g, int64_t n, void* d_series, void* d_tseries) {
    if (int rc = check_grid(g)) return rc;
    if (!g->tws) return fail(TEUK_E_STATE, "teuk_enable_spin_tangent has not been called");
    if (n < 0) return fail(TEUK_E_INVALID_ARG, "n=%lld < 0", (long long)n);
    if (n == 0) return TEUK_OK;
    if (int rc = set_device(g)) return rc;
    const int nr = (int)g->p.nr;
    const int ne = g->p.n_extract;
    double2* series = (ne > 0) ? static_cast<double2*>(d_series) : nullptr;
    double2* tseries = (ne > 0) ? static_cast<double2*>(d_tseries) : nullptr;
    const ExtPoint* ext = g->at<ExtPoint>(g->L.off_ext);
    AdjArgs a = adjoint_args(g);
    a.k.rows = g->tan_rows;
    a.k.n_strips = (nr + kStripCols - 1) / kStripCols;
    a.k.n_chunks = g->tan_chunks;
    // the launches sample their input (row k-1 of a series: the state after
    // step k); the call's last state, or every state when two extraction
    // points share a tile, by a separate pass
    const bool fused = fused_extraction_ok(g, kStripCols, g->tan_rows);
    a.k.n_ext = fused ? ne : 0;
    auto extract = [&](int64_t j) -> int {
        if (series) HIP_TRY(launch_extract(g->u(g->cur), g->L.pitch, ext, ne, series + (j - 1) * ne, g->stream));
        if (tseries) HIP_TRY(launch_extract(g->v(g->vcur), g->L.pitch, ext, ne, tseries + (j - 1) * ne, g->stream));
        return TEUK_OK;
    };
    InLoopCheck chk(g);
    for (int64_t k = 0; k < n; ++k) {
        if (!fused && k > 0)
            if (int rc = extract(k)) return rc;
        double2* su = (series && fused && k > 0) ? series + (k - 1) * ne : nullptr;
        double2* sv = (tseries && fused && k > 0) ? tseries + (k - 1) * ne : nullptr;
        HIP_TRY(launch_spin_tangent(g->u(g->cur), g->v(g->vcur), g->u(1 - g->cur), g->v(1 - g->vcur), su, sv, a,
                                    g->adj_wpb, g->stream));
        g->cur = 1 - g->cur;
        g->vcur = 1 - g->vcur;
        g->steps += 1;
        if (int rc = chk.maybe(g->u(g->cur))) return rc;
    }
    if (int rc = extract(n)) return rc;
    return chk.finish(g->u(g->cur));
}

int teuk_spin_gradient(teuk_grid* g, int64_t n, const void* d_dL_dseries, const void* d_tseries,
                       double* d_dL_da_accum) {
    if (int rc = check_grid(g)) return rc;
    if (n < 0) return fail(TEUK_E_INVALID_ARG, "n=%lld < 0", (long long)n);
    if (!d_dL_da_accum) return fail(TEUK_E_INVALID_ARG, "the dL/da accumulator is NULL");
    const int64_t count = n * g->p.n_extract;
    if (count == 0) return TEUK_OK;
    if (!d_dL_dseries || !d_tseries) return fail(TEUK_E_INVALID_ARG, "series pointers are NULL");
    if (int rc = set_device(g)) return rc;
    HIP_TRY(launch_series_dot(static_cast<const double2*>(d_dL_dseries), static_cast<const double2*>(d_tseries),
                              count, d_dL_da_accum, g->stream));
    return TEUK_OK;
}

/* ---- batched evolutions ------------------------------------------------ */

struct teuk_batch {
    std::vector<teuk_grid*> members;
    std::vector<size_t> ws_off;     // member workspace offsets in the batch workspace
    size_t desc_off = 0;            // descriptor table offset
    size_t ext_off = 0;             // extraction point table offset
    int n_points = 0;               // extraction points of all members
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    int rows = 64, wpb = 4, n_blocks = 0;  // default launch: 64-row tiles, four wavefronts per SIMD
    int total_tiles = 0, total_tiles2 = 0;  // single-step and two-step work lists
    int steps_per_pass = 2;
    int parity = 0;                 // which state buffer of every member is the input
    bool keep = false;              // next states with cache-keeping stores (set by batch_upload)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;  // two launches (parity 0 then 1)
    hipStream_t cap = nullptr;      // private stream the graph is captured on
    int64_t steps = 0;
};

namespace {

size_t batch_layout(const teuk_params* members, int count, std::vector<size_t>* offs, size_t* desc_off,
                    size_t* ext_off = nullptr) {
    size_t o = 0;
    int64_t points = 0;
    for (int k = 0; k < count; ++k) {
        if (offs) offs->push_back(o);
        o += align_up(make_layout(&members[k]).total);
        points += members[k].n_extract;
    }
    if (desc_off) *desc_off = o;
    o += align_up((size_t)count * sizeof(BatchMember));
    if (ext_off) *ext_off = o;
    o += align_up((size_t)std::max<int64_t>(points, 1) * sizeof(BatchExtPoint));
    return o;
}

void batch_drop_graph(teuk_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Descriptor table for the current tile rows; uploaded synchronously.
int batch_upload(teuk_batch* b) {
    std::vector<BatchMember> d(b->members.size());
    int tiles = 0, tiles2 = 0;
    // one launch advances every member: their states share the cache
    size_t states = 0;
    for (const teuk_grid* g : b->members) states += 2 * g->L.state;
    const int keep = states <= kKeepStatesBytes ? 1 : 0;
    b->keep = keep != 0;
    for (size_t k = 0; k < b->members.size(); ++k) {
        teuk_grid* g = b->members[k];
        g->rows = std::min<int>(b->rows, (int)g->p.ntheta);
        StepArgs a = step_args(g);
        BatchMember& M = d[k];
        M.u[0] = g->u(0);
        M.u[1] = g->u(1);
        M.rad = a.rad;
        M.ang = a.ang;
        M.k = a.k;
        M.k.n_ext = 0;
        M.k.keep = keep;
        M.tile_begin = tiles;
        tiles += a.k.n_strips * a.k.n_chunks;
        M.n_strips2 = (a.k.nr + kStripCols2 - 1) / kStripCols2;
        M.tile_begin2 = tiles2;
        tiles2 += M.n_strips2 * a.k.n_chunks;
    }
    b->total_tiles = tiles;
    b->total_tiles2 = tiles2;
    HIP_TRY(hipMemcpyAsync(b->ws + b->desc_off, d.data(), d.size() * sizeof(BatchMember), hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return TEUK_OK;
}

int batch_launch(teuk_batch* b, int parity, bool two, hipStream_t s) {
    const hipError_t e =
        launch_batch(reinterpret_cast<const BatchMember*>(b->ws + b->desc_off), (int)b->members.size(),
                     two ? b->total_tiles2 : b->total_tiles, parity, b->n_blocks, b->wpb, two, b->keep, s);
    return e == hipSuccess ? TEUK_OK : fail(TEUK_E_HIP, "batched step launch failed: %s", hipGetErrorString(e));
}

// Capture two launches (parity 0, then 1; two or four steps) into a graph.  The capture runs on a
// private stream (capturing the caller's stream may not be allowed, e.g. the
// legacy default stream); the graph is launched on the caller's stream.
int batch_capture(teuk_batch* b) {
    if (!b->cap) HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const bool two = b->steps_per_pass == 2;
    const int rc0 = batch_launch(b, 0, two, b->cap);
    const int rc1 = batch_launch(b, 1, two, b->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &graph);
    if (rc0 || rc1 || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(TEUK_E_HIP, "capturing the batched step graph failed: %s", hipGetErrorString(e));
    }
    b->graph = graph;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return TEUK_OK;
}

int batch_check(const teuk_batch* b, int member) {
    if (!b) return fail(TEUK_E_INVALID_ARG, "batch handle is NULL");
    if (member < 0 || member >= (int)b->members.size())
        return fail(TEUK_E_INVALID_ARG, "member %d outside [0, %zu)", member, b->members.size());
    return TEUK_OK;
}

}  // namespace

size_t teuk_batch_workspace_bytes(const teuk_params* members, int32_t count) {
    if (!members || count < 1) {
        fail(TEUK_E_INVALID_ARG, "need count >= 1 members");
        return 0;
    }
    for (int k = 0; k < count; ++k)
        if (validate(&members[k]) != TEUK_OK) return 0;
    return batch_layout(members, count, nullptr, nullptr);
}

int teuk_batch_init(const teuk_params* members, int32_t count, void* hip_stream, void* d_workspace, size_t bytes,
                    teuk_batch** out) {
    if (!members || count < 1 || !out) return fail(TEUK_E_INVALID_ARG, "need members, count >= 1 and out");
    for (int k = 0; k < count; ++k) {
        if (int rc = validate(&members[k])) return rc;
        if (members[k].coef_mode != TEUK_COEF_KERR)
            return fail(TEUK_E_INVALID_ARG, "member %d: batched members use TEUK_COEF_KERR", k);
    }
    if (!d_workspace || reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
        return fail(TEUK_E_WORKSPACE, "batch workspace NULL or not %zu-byte aligned", kAlign);
    teuk_batch* b = new teuk_batch();
    const size_t need = batch_layout(members, count, &b->ws_off, &b->desc_off, &b->ext_off);
    if (bytes < need) {
        delete b;
        return fail(TEUK_E_WORKSPACE, "batch workspace has %zu bytes, needs %zu", bytes, need);
    }
    b->ws = static_cast<char*>(d_workspace);
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    for (int k = 0; k < count; ++k) {
        teuk_grid* g = nullptr;
        const size_t mbytes = make_layout(&members[k]).total;
        if (int rc = teuk_init_grid(&members[k], hip_stream, b->ws + b->ws_off[k], mbytes, &g)) {
            for (teuk_grid* m : b->members) teuk_free(m);
            delete b;
            return rc;
        }
        b->members.push_back(g);
    }
    b->device = b->members[0]->device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess || cus < 1)
        cus = 256;
    // four wavefronts per SIMD: two resident (the two-step kernel's
    // occupancy), and a second round that takes over as the first drains
    b->n_blocks = cus * 16 / b->wpb;
    // the extraction points of all members, in member order
    std::vector<BatchExtPoint> pts;
    for (teuk_grid* g : b->members)
        for (const ExtPoint& e : g->ext) {
            BatchExtPoint q{};
            q.u[0] = g->u(0);
            q.u[1] = g->u(1);
            q.pitch = g->L.pitch;
            q.e = e;
            pts.push_back(q);
        }
    b->n_points = (int)pts.size();
    hipError_t e = hipSuccess;
    if (!pts.empty()) {
        e = hipMemcpyAsync(b->ws + b->ext_off, pts.data(), pts.size() * sizeof(BatchExtPoint), hipMemcpyHostToDevice,
                           b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    }
    if (e != hipSuccess) {
        for (teuk_grid* m : b->members) teuk_free(m);
        delete b;
        return fail(TEUK_E_HIP, "uploading the extraction points: %s", hipGetErrorString(e));
    }
    if (int rc = batch_upload(b)) {
        for (teuk_grid* m : b->members) teuk_free(m);
        delete b;
        return rc;
    }
    *out = b;
    return TEUK_OK;
}

int teuk_batch_set_initial_data(teuk_batch* b, int32_t member, const void* d_phi, const void* d_pi) {
    if (int rc = batch_check(b, member)) return rc;
    if (!d_phi || !d_pi) return fail(TEUK_E_INVALID_ARG, "initial data pointers are NULL");
    teuk_grid* g = b->members[member];
    if (int rc = set_device(g)) return rc;
    const int nr = (int)g->p.nr, nth = (int)g->p.ntheta;
    HIP_TRY(launch_import(static_cast<const double2*>(d_phi), g->u(b->parity), 0, nr, nth, g->L.pitch, g->stream));
    HIP_TRY(launch_import(static_cast<const double2*>(d_pi), g->u(b->parity), 1, nr, nth, g->L.pitch, g->stream));
    g->cur = b->parity;
    g->steps = 0;
    return TEUK_OK;
}

int teuk_batch_get_state(teuk_batch* b, int32_t member, void* d_phi, void* d_pi) {
    if (int rc = batch_check(b, member)) return rc;
    return teuk_get_state(b->members[member], d_phi, d_pi);
}

int teuk_batch_step_n(teuk_batch* b, int64_t n) {
    if (int rc = batch_check(b, 0)) return rc;
    if (n < 0) return fail(TEUK_E_INVALID_ARG, "n=%lld < 0", (long long)n);
    if (n == 0) return TEUK_OK;
    if (int rc = set_device(b->members[0])) return rc;
    // launches of `per` steps each flip the parity; whole graphs (two
    // launches) start from parity 0; an odd last step runs alone
    const int per = b->steps_per_pass;
    int64_t left = n;
    while (left > 0) {
        if (b->parity == 0 && left >= 2 * per) {
            if (!b->exec)  // captured once per launch configuration
                if (int rc = batch_capture(b)) return rc;
            for (; left >= 2 * per; left -= 2 * per) HIP_TRY(hipGraphLaunch(b->exec, b->stream));
            continue;
        }
        const bool two = left >= per && per == 2;
        if (int rc = batch_launch(b, b->parity, two, b->stream)) return rc;
        b->parity = 1 - b->parity;
        left -= two ? 2 : 1;
    }
    b->steps += n;
    for (teuk_grid* g : b->members) {
        g->cur = b->parity;
        g->steps += n;
    }
    return TEUK_OK;
}

int teuk_batch_set_launch(teuk_batch* b, int32_t rows_per_tile, int32_t waves_per_block, int32_t n_blocks) {
    if (int rc = batch_check(b, 0)) return rc;
    if (rows_per_tile < 1 || rows_per_tile > 4096)
        return fail(TEUK_E_INVALID_ARG, "rows_per_tile=%d outside [1, 4096]", rows_per_tile);
    if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4 && waves_per_block != 8)
        return fail(TEUK_E_INVALID_ARG, "waves_per_block=%d not in {1, 2, 4, 8}", waves_per_block);
    if (n_blocks < 1 || n_blocks > (1 << 20)) return fail(TEUK_E_INVALID_ARG, "n_blocks=%d out of range", n_blocks);
    if (int rc = set_device(b->members[0])) return rc;
    HIP_TRY(hipStreamSynchronize(b->stream));  // in-flight launches read the old descriptors
    batch_drop_graph(b);
    b->rows = rows_per_tile;
    b->wpb = waves_per_block;
    b->n_blocks = n_blocks;
    return batch_upload(b);
}

int teuk_batch_set_steps_per_pass(teuk_batch* b, int32_t steps_per_pass) {
    if (int rc = batch_check(b, 0)) return rc;
    if (steps_per_pass != 1 && steps_per_pass != 2)
        return fail(TEUK_E_INVALID_ARG, "steps_per_pass=%d not in {1, 2}", steps_per_pass);
    if (steps_per_pass == b->steps_per_pass) return TEUK_OK;
    if (int rc = set_device(b->members[0])) return rc;
    HIP_TRY(hipStreamSynchronize(b->stream));
    batch_drop_graph(b);
    b->steps_per_pass = steps_per_pass;
    return TEUK_OK;
}

int teuk_batch_get_launch(const teuk_batch* b, int32_t* rows_per_tile, int32_t* waves_per_block,
                          int32_t* n_blocks) {
    if (int rc = batch_check(b, 0)) return rc;
    if (rows_per_tile) *rows_per_tile = b->rows;
    if (waves_per_block) *waves_per_block = b->wpb;
    if (n_blocks) *n_blocks = b->n_blocks;
    return TEUK_OK;
}

int teuk_batch_extract(teuk_batch* b, void* d_out) {
    if (int rc = batch_check(b, 0)) return rc;
    if (b->n_points == 0) return fail(TEUK_E_STATE, "no member has extraction points");
    if (!d_out) return fail(TEUK_E_INVALID_ARG, "output pointer is NULL");
    if (int rc = set_device(b->members[0])) return rc;
    HIP_TRY(launch_batch_extract(reinterpret_cast<const BatchExtPoint*>(b->ws + b->ext_off), b->n_points, b->parity,
                                 static_cast<double2*>(d_out), b->stream));
    return TEUK_OK;
}

int32_t teuk_batch_n_extract(const teuk_batch* b) { return b ? b->n_points : -1; }

int teuk_assemble_modes(int64_t n_samples, int32_t n_modes, const int32_t* h_m, int32_t n_obs, const double* h_phi,
                        const double* h_r, const void* d_samples, void* d_psi, void* hip_stream) {
    if (n_samples < 0) return fail(TEUK_E_INVALID_ARG, "n_samples=%lld < 0", (long long)n_samples);
    if (n_modes < 1 || n_modes > kMaxModes) return fail(TEUK_E_INVALID_ARG, "n_modes=%d outside [1, %d]", n_modes, kMaxModes);
    if (n_obs < 1 || n_obs > kMaxObservers) return fail(TEUK_E_INVALID_ARG, "n_obs=%d outside [1, %d]", n_obs, kMaxObservers);
    if (!h_m || !h_phi || !h_r) return fail(TEUK_E_INVALID_ARG, "mode or observer arrays are NULL");
    if (n_samples > 0 && (!d_samples || !d_psi)) return fail(TEUK_E_INVALID_ARG, "device pointers are NULL");
    AssembleArgs a{};
    a.n_modes = n_modes;
    a.n_obs = n_obs;
    for (int j = 0; j < n_modes; ++j) a.m[j] = h_m[j];
    for (int o = 0; o < n_obs; ++o) {
        if (!std::isfinite(h_phi[o]) || !std::isfinite(h_r[o]) || !(h_r[o] > 0.0))
            return fail(TEUK_E_INVALID_ARG, "observer %d: need finite phi and r > 0", o);
        a.phi[o] = h_phi[o];
        a.r3[o] = h_r[o] * h_r[o] * h_r[o];
    }
    HIP_TRY(launch_assemble(a, n_samples, static_cast<const double2*>(d_samples), static_cast<double2*>(d_psi),
                            reinterpret_cast<hipStream_t>(hip_stream)));
    return TEUK_OK;
}

int64_t teuk_batch_total_points(const teuk_batch* b) {
    if (!b) return -1;
    int64_t n = 0;
    for (const teuk_grid* g : b->members) n += g->p.nr * g->p.ntheta;
    return n;
}

int teuk_batch_free(teuk_batch* b) {
    if (!b) return TEUK_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (teuk_grid* g : b->members) teuk_free(g);
    delete b;
    if (e != hipSuccess) return fail(TEUK_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return TEUK_OK;
}

int teuk_free(teuk_grid* g) {
    if (!g) return TEUK_OK;
    hipError_t e = hipStreamSynchronize(g->stream);
    delete g;
    if (e != hipSuccess) return fail(TEUK_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return TEUK_OK;
}

}  // extern "C"
