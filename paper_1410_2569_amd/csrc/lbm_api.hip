// lbm_api.hip -- C ABI of liblbm (declared in include/lbm.h): parameter validation, workspace
// carving, stream-ordered launches of the kernels in lbm_kernels.hip, observables post-processing
// and the Carnahan-Starling Maxwell construction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.h"

using lbm::KParams;

struct lbm_ctx {
    lbm_params p;
    KParams kp;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    double* g[2];
    double* psi;
    double* gw;
    double* part;
    double* fin;
    int cur;
    int64_t step;
    int schedule;
    int tile;
    int tile2;  // output tile of the two-step kernel
    // last lbm_forward_ckpt: where it started, its length and checkpoint interval
    int64_t adj_start, adj_nsteps;
    int32_t adj_K;
    const void* adj_ws;
    // lbm_backward recomputes the next segment on a stream of its own (default priority) while
    // the caller's stream runs the current one in reverse; created on first use
    hipStream_t aux = nullptr;
    hipEvent_t ev_start = nullptr, ev_rc[2] = {}, ev_free[2] = {};
    std::string err;
};

namespace {

constexpr size_t kAlign = 256;

// Message of the last failed lbm_create* / lbm_batch_create* on this thread (no handle exists
// then); returned by lbm_last_error(NULL) and lbm_batch_last_error(NULL).
thread_local std::string g_create_err;

int create_fail(int code, const char* what, hipError_t e) {
    g_create_err = std::string(what) + ": " + hipGetErrorString(e);
    return code;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Every copy between host and device memory is one contiguous synchronous transfer made after
// the stream's queued work has completed: pitched fields are packed or unpacked on the device
// (k_repack) next to a dense staging copy. The host buffers of this API are ordinary pageable
// memory; a synchronous copy is complete when it returns, and the preceding synchronisation
// orders it after the stream's kernels (every kernel enqueued later sees it). No strided (2D)
// copy is used: with a kernel tracer attached those have been observed not to deliver their data.
hipError_t host_copy(hipStream_t s, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    return hipMemcpy(dst, src, bytes, kind);
}

// Dense host array [planes][rows][nx] -> device field with rows `pitch` and planes `plane`
// doubles apart, through `stage` (device memory of planes * rows * nx doubles, free here).
hipError_t upload_field(hipStream_t s, const double* host, int planes, int rows, int nx,
                        double* stage, double* dst, long long plane, int pitch) {
    hipError_t e = host_copy(s, stage, host, sizeof(double) * planes * rows * nx,
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    return lbm::launch_repack(stage, (long long)rows * nx, nx, dst, plane, pitch, nx, rows, planes,
                              s);
}

// Device field (rows `pitch`, planes `plane` apart) -> dense host array [planes][rows][nx],
// through `stage` (device memory of planes * rows * nx doubles, free here).
hipError_t download_field(hipStream_t s, const double* src, long long plane, int pitch,
                          int planes, int rows, int nx, double* stage, double* host) {
    hipError_t e = lbm::launch_repack(src, plane, pitch, stage, (long long)rows * nx, nx, nx, rows,
                                      planes, s);
    if (e != hipSuccess) return e;
    return host_copy(s, host, stage, sizeof(double) * planes * rows * nx, hipMemcpyDeviceToHost);
}

struct Layout {
    int pitch;
    long long plane;  // doubles
    size_t off_g0, off_g1, off_psi, off_gw, off_links, off_part, off_fin, total;
};

bool is_mask(const lbm_params* p) { return p->walls == LBM_WALLS_MASK; }
int y_lo_of(const lbm_params* p) { return (p->walls == 1 || p->walls == 2) ? 1 : 0; }
int y_hi_of(const lbm_params* p) { return (p->walls == 1 || p->walls == 2) ? p->ny - 2 : p->ny - 1; }

Layout layout_of(const lbm_params* p) {
    Layout L;
    L.pitch = (int)align_up((size_t)p->nx, 32);
    L.plane = (long long)p->ny * L.pitch;
    size_t fbytes = align_up((size_t)(9 * L.plane) * sizeof(double), kAlign);
    size_t o = 0;
    L.off_g0 = o; o += fbytes;
    L.off_g1 = o; o += fbytes;
    L.off_psi = o; o += align_up((size_t)L.plane * sizeof(double), kAlign);
    // G_w: two wall rows, or one value per node with a solid mask (plus its link words)
    L.off_gw = o; o += align_up((size_t)(is_mask(p) ? p->ny : 2) * L.pitch * sizeof(double), kAlign);
    L.off_links = o;
    if (is_mask(p)) o += align_up((size_t)L.plane * sizeof(unsigned short), kAlign);
    KParams tmp{};
    tmp.nx = p->nx; tmp.ny = p->ny;
    tmp.y_lo = y_lo_of(p); tmp.y_hi = y_hi_of(p);
    L.off_part = o; o += align_up((size_t)lbm::obs_blocks(tmp) * lbm::OBS_NQ * sizeof(double), kAlign);
    L.off_fin = o; o += align_up(32 * sizeof(double), kAlign);
    L.total = o;
    return L;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Validation without any HIP call. Returns LBM_OK or an error code with a message.
int validate(const lbm_params* p, std::string* msg) {
    auto bad = [&](const char* m) { if (msg) *msg = m; return LBM_E_INVAL; };
    if (!p) return bad("null parameter block");
    if (p->abi_version != LBM_ABI_VERSION) {
        if (msg) *msg = "abi_version mismatch";
        return LBM_E_ABI;
    }
    if (p->walls < LBM_PERIODIC || p->walls > LBM_WALLS_MASK) return bad("walls must be 0, 1, 2 or 3");
    if (p->walls == LBM_WALLS_MASK && p->ghost_psi != 0)
        return bad("a solid mask has no ghost layer: ghost_psi must be 0");
    if (p->ghost_psi != 0 && p->ghost_psi != 1) return bad("ghost_psi must be 0 or 1");
    if (p->nx < 3) return bad("nx must be >= 3");
    if (p->ny < (y_lo_of(p) ? 4 : 3)) return bad("ny must be >= 4 with walls (>= 3 without)");
    if ((long long)p->nx * p->ny > (1LL << 31)) return bad("lattice too large");
    if (p->eos != LBM_EOS_CS && p->eos != LBM_EOS_PIECEWISE) return bad("unknown eos");
    if (p->wall_force < LBM_WALL_RHO || p->wall_force > LBM_WALL_MODPSI) return bad("unknown wall_force");
    if (p->reserved != 0) return bad("reserved must be 0");
    if (!(std::isfinite(p->G) && p->G < 0.0)) return bad("G must be negative");
    if (!std::isfinite(p->sigma)) return bad("sigma must be finite");
    const double rates[5] = {p->s_rho, p->s_e, p->s_zeta, p->s_j, p->s_q};
    for (double s : rates)
        if (!(std::isfinite(s) && s > 0.0 && s < 2.0)) return bad("relaxation rates must lie in (0, 2)");
    if (!(std::isfinite(p->tau_l) && p->tau_l > 0.5 && std::isfinite(p->tau_v) && p->tau_v > 0.5))
        return bad("tau_l and tau_v must exceed 1/2");
    if (!(finite_pos(p->rho_v) && finite_pos(p->rho_l) && p->rho_l > p->rho_v))
        return bad("need rho_l > rho_v > 0");
    if (p->eos == LBM_EOS_CS) {
        if (!(finite_pos(p->a) && finite_pos(p->b) && finite_pos(p->R) && finite_pos(p->T)))
            return bad("Carnahan-Starling a, b, R, T must be positive");
    } else {
        if (!(finite_pos(p->rho1) && p->rho2 > p->rho1 && std::isfinite(p->rho2) &&
              std::isfinite(p->th_v) && std::isfinite(p->th_m) && std::isfinite(p->th_l)))
            return bad("piecewise EOS needs 0 < rho1 < rho2 and finite slopes");
    }
    return LBM_OK;
}

KParams kparams_of(const lbm_params* p, const Layout& L) {
    KParams k{};
    k.nx = p->nx; k.ny = p->ny; k.pitch = L.pitch; k.plane = L.plane;
    k.walls = p->walls; k.ghost = p->ghost_psi; k.eos = p->eos; k.wall_force = p->wall_force;
    k.wet = p->walls == LBM_WALLS_WET_NODE ? 1 : 0;
    k.mask = is_mask(p) ? 1 : 0;
    k.y_lo = y_lo_of(p);
    k.y_hi = y_hi_of(p);
    k.RT = p->R * p->T; k.a = p->a; k.b4 = p->b / 4.0;
    k.rho1 = p->rho1; k.rho2 = p->rho2; k.th_v = p->th_v; k.th_m = p->th_m; k.th_l = p->th_l;
    k.p1 = p->rho1 * p->th_v;
    k.p2 = k.p1 + (p->rho2 - p->rho1) * p->th_m;
    k.two_over_G = 2.0 / p->G;
    k.rho_mid = 0.5 * (p->rho_l + p->rho_v);
    k.negG = -p->G;
    const double tau_e = 1.0 / p->s_e, tau_z = 1.0 / p->s_zeta;
    k.c_sig_e = 12.0 * p->sigma * p->G * p->G / (tau_e - 0.5);
    k.c_sig_z = 12.0 * p->sigma * p->G * p->G / (tau_z - 0.5);
    k.s_e = p->s_e; k.s_z = p->s_zeta; k.s_j = p->s_j; k.s_q = p->s_q;
    k.h_e = 1.0 - 0.5 * p->s_e; k.h_z = 1.0 - 0.5 * p->s_zeta;
    k.h_j = 1.0 - 0.5 * p->s_j; k.h_q = 1.0 - 0.5 * p->s_q;
    const double nu_l = (p->tau_l - 0.5) / 3.0, nu_v = (p->tau_v - 0.5) / 3.0;
    k.nu_v = nu_v; k.dnu = nu_l - nu_v; k.rho_v = p->rho_v;
    k.inv_drho = 1.0 / (p->rho_l - p->rho_v);
    k.visc_const = p->tau_l == p->tau_v ? 1 : 0;
    k.s_nu_c = 1.0 / (3.0 * nu_v + 0.5);
    return k;
}

int fail(lbm_ctx* c, int code, const std::string& m) {
    if (c) c->err = m;
    return code;
}

int hip_fail(lbm_ctx* c, hipError_t e, const char* where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(c, LBM_E_HIP, m);
}

// -------------------------------------------------------------------------------------------
// Carnahan-Starling thermodynamics, closed forms:
//   p(rho) = rho R T Z(eta) - a rho^2,  Z = (1 + eta + eta^2 - eta^3)/(1 - eta)^3, eta = b rho/4
//   Phi(rho) = integral p / rho^2 d rho = R T [ln eta + (4 eta - 3 eta^2)/(1 - eta)^2] - a rho
//   equal area: Phi(rho_l) - Phi(rho_v) = p0 (1/rho_v - 1/rho_l)
// -------------------------------------------------------------------------------------------
struct CS {
    double a, b, RT;
    double p(double r) const {
        double e = b * r / 4.0, om = 1.0 - e;
        return r * RT * (1.0 + e + e * e - e * e * e) / (om * om * om) - a * r * r;
    }
    double dp(double r) const {
        double e = b * r / 4.0, om = 1.0 - e;
        return RT * (1.0 + 4.0 * e + 4.0 * e * e - 4.0 * e * e * e + e * e * e * e) /
                   (om * om * om * om) - 2.0 * a * r;
    }
    double Phi(double r) const {
        double e = b * r / 4.0, om = 1.0 - e;
        return RT * (std::log(e) + (4.0 * e - 3.0 * e * e) / (om * om)) - a * r;
    }
};

template <class F>
double bisect(F&& fn, double lo, double hi, int iters = 200) {
    double flo = fn(lo);
    for (int i = 0; i < iters; ++i) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        double fm = fn(mid);
        if ((fm > 0) == (flo > 0)) { lo = mid; flo = fm; } else { hi = mid; }
    }
    return 0.5 * (lo + hi);
}

int maxwell_cs_impl(double a, double b, double R, double T, double* rv, double* rl, double* p0) {
    CS cs{a, b, R * T};
    const double top = 4.0 / b;
    // spinodals: sign changes of dp on a fine logarithmic grid in (0, 4/b)
    double sp[2];
    int ns = 0;
    const int n = 20000;
    double prev_r = top * 1e-9, prev = cs.dp(prev_r);
    for (int i = 1; i <= n && ns < 2; ++i) {
        double r = top * std::pow(10.0, -9.0 + 9.0 * i / n) * (1.0 - 1e-9);
        double d = cs.dp(r);
        if ((d > 0) != (prev > 0)) {
            sp[ns++] = bisect([&](double x) { return cs.dp(x); }, prev_r, r);
        }
        prev = d; prev_r = r;
    }
    if (ns < 2) return LBM_E_INVAL;
    const double s1 = sp[0], s2 = sp[1];
    double plo = std::max(cs.p(s2), 0.0), phi = cs.p(s1);
    if (!(phi > plo)) return LBM_E_INVAL;
    auto branches = [&](double pp, double* v, double* l) {
        *v = bisect([&](double x) { return cs.p(x) - pp; }, 1e-300, s1);
        *l = bisect([&](double x) { return cs.p(x) - pp; }, s2, top * (1.0 - 1e-12));
    };
    auto area = [&](double pp) {
        double v, l;
        branches(pp, &v, &l);
        return (cs.Phi(l) - cs.Phi(v)) - pp * (1.0 / v - 1.0 / l);
    };
    double lo = plo + (phi - plo) * 1e-12, hi = phi - (phi - plo) * 1e-12;
    double pm = bisect(area, lo, hi);
    branches(pm, rv, rl);
    if (p0) *p0 = pm;
    return LBM_OK;
}

struct AdjLayout {
    int64_t nck;
    size_t fbytes, pbytes, rbytes;
    size_t off_ck, off_seg, off_a, off_q, off_p0, off_dpsi, off_rv, off_gg, off_part, off_fin,
        total;
};

// Adjoint workspace: the checkpoints, the segment store (segs of them, K states each), then the
// adjoint quantities of two consecutive reverse steps (a: 9 planes, q: 2 planes, p0, psi', r: 4
// rows, each twice) and the G_w gradient; the adjoint part is cleared at the start of every
// backward pass. A single lattice keeps two segment stores (one recomputed while the other is
// reversed), an ensemble instance one.
AdjLayout adj_layout_of(const lbm_params* p, int64_t nsteps, int32_t K, int segs) {
    AdjLayout A;
    Layout L = layout_of(p);
    A.nck = (nsteps + K - 1) / K;
    A.fbytes = align_up((size_t)(9 * L.plane) * sizeof(double), kAlign);
    A.pbytes = align_up((size_t)L.plane * sizeof(double), kAlign);
    A.rbytes = align_up((size_t)4 * L.pitch * sizeof(double), kAlign);
    KParams tmp{};
    tmp.nx = p->nx; tmp.ny = p->ny;
    tmp.y_lo = p->walls ? 1 : 0; tmp.y_hi = p->walls ? p->ny - 2 : p->ny - 1;
    size_t o = 0;
    A.off_ck = o; o += (size_t)A.nck * A.fbytes;
    A.off_seg = o; o += (size_t)segs * K * A.fbytes;
    A.off_a = o; o += 2 * A.fbytes;
    A.off_q = o; o += 4 * A.pbytes;
    A.off_p0 = o; o += 2 * A.pbytes;
    A.off_dpsi = o; o += 2 * A.pbytes;
    A.off_rv = o; o += 2 * A.rbytes;
    A.off_gg = o; o += align_up((size_t)2 * L.pitch * sizeof(double), kAlign);
    A.off_part = o; o += align_up((size_t)lbm::loss_blocks(tmp) * 3 * sizeof(double), kAlign);
    A.off_fin = o; o += kAlign;
    A.total = o;
    return A;
}

}  // namespace

// ---- allocation-free observables ------------------------------------------------------------
// Scratch of lbm_observables_of_state: a fixed device array of the library (every GPU the library
// runs on holds one until the process ends). In host code `scratch` names a host-side stand-in,
// not device memory: kernels and copies only ever get the per-device address that
// hipGetSymbolAddress returns.
constexpr size_t kStaticScratchBytes = size_t(24) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device, looked up once per device.
hipError_t static_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

// =============================================================================================
extern "C" {

const char* lbm_strerror(int code) {
    switch (code) {
        case LBM_OK: return "ok";
        case LBM_E_INVAL: return "invalid argument";
        case LBM_E_SIZE: return "buffer too small";
        case LBM_E_HIP: return "HIP runtime error";
        case LBM_E_NONFINITE: return "non-finite state";
        case LBM_E_ABI: return "ABI version mismatch";
        case LBM_E_STATE: return "state does not match context";
        default: return "unknown error";
    }
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

int lbm_maxwell_cs(double a, double b, double R, double T, double* rho_v, double* rho_l,
                   double* p0) {
    if (!rho_v || !rho_l) return LBM_E_INVAL;
    if (!(finite_pos(a) && finite_pos(b) && finite_pos(R) && finite_pos(T))) return LBM_E_INVAL;
    return maxwell_cs_impl(a, b, R, T, rho_v, rho_l, p0);
}

int lbm_cs_temperature(double a, double b, double R, double ratio, double* T) {
    if (!T || !(finite_pos(a) && finite_pos(b) && finite_pos(R)) || !(ratio > 1.0))
        return LBM_E_INVAL;
    // critical temperature bracket: scan down from a high T until two-phase
    double Tc_hi = 2.0 * a / (b * R), Tlo = 0.0, Thi = 0.0;
    double v, l;
    for (double t = Tc_hi; t > 1e-6 * Tc_hi; t *= 0.98) {
        if (maxwell_cs_impl(a, b, R, t, &v, &l, nullptr) == LBM_OK && l / v > 1.0001) { Thi = t; break; }
    }
    if (Thi == 0.0) return LBM_E_INVAL;
    Tlo = Thi;
    for (int i = 0; i < 200; ++i) {
        Tlo *= 0.95;
        if (maxwell_cs_impl(a, b, R, Tlo, &v, &l, nullptr) != LBM_OK) return LBM_E_INVAL;
        if (l / v > ratio) break;
    }
    auto g = [&](double t) {
        double vv, ll;
        if (maxwell_cs_impl(a, b, R, t, &vv, &ll, nullptr) != LBM_OK) return 1.0;
        return std::log(ll / vv) - std::log(ratio);
    };
    *T = bisect(g, Tlo, Thi, 100);
    return LBM_OK;
}

// Spinodal densities of the piecewise-linear EOS, Eq. (15), for given coexistence densities
// (Sec. III). With p0 = rho_v th_v, mechanical equilibrium p(rho_l) = p0 is linear in (rho1, rho2)
// and fixes rho2(rho1); chemical equilibrium is the equal-area rule
//   sum over the three linear pieces p = A + th rho of  (A - p0)(1/lo - 1/hi) + th ln(hi/lo) = 0,
// the closed-form integral of (p - p0)/rho^2 on [lo, hi]. The root in rho1 is bracketed on a
// logarithmic scan of (rho_v, rho_l) and bisected.
int lbm_piecewise_spinodals(double rho_v, double rho_l, double th_v, double th_m, double th_l,
                            double* rho1, double* rho2) {
    if (!rho1 || !rho2 || !(finite_pos(rho_v) && std::isfinite(rho_l) && rho_l > rho_v) ||
        !(std::isfinite(th_v) && std::isfinite(th_m) && std::isfinite(th_l)) || !(th_m < th_l))
        return LBM_E_INVAL;
    const double p0 = rho_v * th_v;
    auto r2_of = [&](double r1) { return (p0 - r1 * (th_v - th_m) - th_l * rho_l) / (th_m - th_l); };
    auto piece = [&](double A, double th, double lo, double hi) {
        return (A - p0) * (1.0 / lo - 1.0 / hi) + th * std::log(hi / lo);
    };
    auto chem = [&](double r1) {
        const double r2 = r2_of(r1);
        const double A2 = r1 * (th_v - th_m);
        const double A3 = A2 + r2 * (th_m - th_l);
        return piece(0.0, th_v, rho_v, r1) + piece(A2, th_m, r1, r2) + piece(A3, th_l, r2, rho_l);
    };
    auto valid = [&](double r1) { const double r2 = r2_of(r1); return r1 < r2 && r2 < rho_l; };
    const int n = 4000;
    const double lr = std::log(rho_l / rho_v);
    double prev = rho_v * (1.0 + 1e-12), fprev = NAN;
    for (int k = 1; k <= n; ++k) {
        const double r1 = rho_v * std::exp(lr * k / n);
        if (!valid(r1)) { fprev = NAN; prev = r1; continue; }
        const double fc = chem(r1);
        if (std::isfinite(fprev) && (fc > 0) != (fprev > 0)) {
            const double r = bisect(chem, prev, r1);
            *rho1 = r;
            *rho2 = r2_of(r);
            return LBM_OK;
        }
        prev = r1;
        fprev = fc;
    }
    return LBM_E_INVAL;
}

// p_EOS(rho) on the host: Carnahan-Starling or Eq. (15). With psi = sqrt(2 (p - rho/3)/G) the
// bulk pressure of Eq. (8), rho c_s^2 + G c^2 psi^2 / 2, equals it.
// p_EOS(rho) on the host (Carnahan-Starling or Eq. 15); false outside the EOS domain.
static bool host_pressure(const lbm_params* p, double rho, double* out) {
    if (!std::isfinite(rho) || rho < 0.0) return false;
    if (p->eos == LBM_EOS_CS) {
        const double e = p->b * rho / 4.0, om = 1.0 - e;
        if (!(om > 0.0)) return false;
        *out = rho * p->R * p->T * (1.0 + e + e * e - e * e * e) / (om * om * om) - p->a * rho * rho;
    } else {
        const double p1 = p->rho1 * p->th_v, p2 = p1 + (p->rho2 - p->rho1) * p->th_m;
        *out = rho <= p->rho1 ? rho * p->th_v
             : (rho <= p->rho2 ? p1 + (rho - p->rho1) * p->th_m : p2 + (rho - p->rho2) * p->th_l);
    }
    return std::isfinite(*out);
}

// The pseudopotential psi = sqrt(2 (p_EOS(rho) - rho/3) / G) exists at rho (non-negative radicand).
static bool psi_defined(const lbm_params* p, double rho) {
    double pr;
    if (!host_pressure(p, rho, &pr)) return false;
    const double rad = 2.0 * (pr - rho / 3.0) / p->G;
    return std::isfinite(rad) && rad >= 0.0;
}

int lbm_pressure(const lbm_params* p, double rho, double* out) {
    if (!out || validate(p, nullptr) != LBM_OK) return LBM_E_INVAL;
    return host_pressure(p, rho, out) ? LBM_OK : LBM_E_INVAL;
}

int lbm_workspace_size(const lbm_params* p, size_t* bytes) {
    if (!bytes) return LBM_E_INVAL;
    int rc = validate(p, nullptr);
    if (rc) return rc;
    *bytes = layout_of(p).total;
    return LBM_OK;
}

// Link words of a solid mask: bit 0 = node solid, bit a = node x - e_a solid (x, y periodic).
static std::vector<unsigned short> mask_links(const lbm_params* p, const uint8_t* solid, int pitch) {
    static const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    std::vector<unsigned short> lk((size_t)p->ny * pitch, 1);  // padding columns: solid
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            unsigned short w = 0;
            for (int a = 0; a < 9; ++a) {
                const int xs = ((x - ex[a]) % p->nx + p->nx) % p->nx;
                const int ys = ((y - ey[a]) % p->ny + p->ny) % p->ny;
                if (solid[(size_t)ys * p->nx + xs]) w |= (unsigned short)(1u << a);
            }
            lk[(size_t)y * pitch + x] = w;
        }
    return lk;
}

// Droplet description checks: count in 1..64, finite centres, positive radii and width, jitter in
// [0, 1) (so that every generated density stays positive).
static bool droplets_ok(const lbm_droplets* d) {
    if (!d || d->count < 1 || d->count > LBM_MAX_DROPLETS || d->reserved != 0) return false;
    if (!finite_pos(d->width) || !std::isfinite(d->jitter) || d->jitter < 0.0 || d->jitter >= 1.0)
        return false;
    for (int k = 0; k < d->count; ++k)
        if (!std::isfinite(d->x0[k]) || !std::isfinite(d->y0[k]) || !finite_pos(d->radius[k]))
            return false;
    return true;
}

static uint64_t splitmix64_host(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One of rho0_host (host density field) and drops (droplets generated on the device) is given.
static int create_impl(const lbm_params* p, const uint8_t* solid, const double* gw_host,
                       const double* rho0_host, const lbm_droplets* drops, void* d_ws,
                       size_t ws_bytes, void* stream, lbm_ctx** out) {
    if (!out) return LBM_E_INVAL;
    *out = nullptr;
    std::string msg;
    int rc = validate(p, &msg);
    if (rc) return rc;
    if (!rho0_host == !drops || !d_ws) return LBM_E_INVAL;
    if (drops && (solid || !droplets_ok(drops))) return LBM_E_INVAL;
    if (p->walls && !gw_host) return LBM_E_INVAL;
    if (is_mask(p) != (solid != nullptr)) return LBM_E_INVAL;
    if (rho0_host) {
        // every fluid density positive, finite and inside the pseudopotential's domain
        long long nfluid = 0;
        for (long long i = 0; i < (long long)p->nx * p->ny; ++i) {
            const int y = (int)(i / p->nx);
            if (solid ? solid[i] != 0 : (y < y_lo_of(p) || y > y_hi_of(p))) continue;
            if (!finite_pos(rho0_host[i]) || !psi_defined(p, rho0_host[i])) return LBM_E_INVAL;
            ++nfluid;
        }
        if (nfluid == 0) return LBM_E_INVAL;
    } else {
        // the droplet profiles lie between rho_v (1 - jitter) and rho_l (1 + jitter)
        const double lo = p->rho_v * (1.0 - drops->jitter), hi = p->rho_l * (1.0 + drops->jitter);
        for (int k = 0; k <= 1024; ++k)
            if (!psi_defined(p, lo + (hi - lo) * k / 1024.0)) return LBM_E_INVAL;
    }
    const int gw_rows = solid ? p->ny : 2;
    if (gw_host)
        for (long long i = 0; i < (long long)gw_rows * p->nx; ++i)
            if (!std::isfinite(gw_host[i])) return LBM_E_INVAL;
    Layout L = layout_of(p);
    if (ws_bytes < L.total) return LBM_E_SIZE;
    if (((uintptr_t)d_ws) % kAlign) return LBM_E_INVAL;

    (void)hipGetLastError();  // report only errors of this call
    lbm_ctx* c = new lbm_ctx();
    c->p = *p;
    c->kp = kparams_of(p, L);
    c->stream = (hipStream_t)stream;
    c->ws = (char*)d_ws;
    c->ws_bytes = ws_bytes;
    c->g[0] = (double*)(c->ws + L.off_g0);
    c->g[1] = (double*)(c->ws + L.off_g1);
    c->psi = (double*)(c->ws + L.off_psi);
    c->gw = (double*)(c->ws + L.off_gw);
    c->part = (double*)(c->ws + L.off_part);
    c->fin = (double*)(c->ws + L.off_fin);
    c->cur = 0;
    c->step = 0;
    c->schedule = 2;  // two steps per launch (bit-identical to single steps, fastest)
    c->tile = 1;
    // 64 x 8 output tiles, or the wide 32 x 4 workgroups on lattices of at most 384 such tiles
    // (about 1.5 per compute unit), which a launch runs in one round of short chains. Measured
    // per two-step launch (one MI355X; 64x8 / 64x4 / wide 32x4): 128x64 7.24 / 6.54 / 5.55 us,
    // 256x128 7.35 / 6.74 / 5.78, 384x192 7.76 / 8.58 / 7.98, 512x256 8.39 / 9.44 / 10.56.
    c->tile2 = ((p->nx + 31) / 32) * ((y_hi_of(p) - y_lo_of(p) + 4) / 4) <= 384 ? 7 : 0;
    c->adj_start = -1;
    c->adj_nsteps = 0;
    c->adj_K = 0;
    c->adj_ws = nullptr;

    hipStream_t s = c->stream;
    hipError_t e;
    if ((e = lbm::launch_zero(c->ws, L.total, s)) != hipSuccess) { delete c; return create_fail(LBM_E_HIP, "create: workspace clear", e); }
    // host arrays are staged in the second population buffer, which the first step overwrites
    if (gw_host) {
        e = upload_field(s, gw_host, 1, gw_rows, p->nx, c->g[1], c->gw, 0, L.pitch);
        if (e != hipSuccess) { delete c; return create_fail(LBM_E_HIP, "create: G_w copy", e); }
    }
    if (solid) {
        std::vector<unsigned short> lk = mask_links(p, solid, L.pitch);
        unsigned short* d_links = (unsigned short*)(c->ws + L.off_links);
        e = host_copy(s, d_links, lk.data(), lk.size() * sizeof(unsigned short),
                      hipMemcpyHostToDevice);
        if (e != hipSuccess) { delete c; return create_fail(LBM_E_HIP, "create: links copy", e); }
        c->kp.links = d_links;
        c->kp.gwn = c->gw;
    }
    // rho0 into plane 1 of the second population buffer, then the first buffer built from it
    double* rho0 = c->g[1] + L.plane;
    if (rho0_host) {
        e = upload_field(s, rho0_host, 1, p->ny, p->nx, c->g[1], rho0, 0, L.pitch);
        if (e != hipSuccess) { delete c; return create_fail(LBM_E_HIP, "create: rho0 copy", e); }
    } else {
        lbm::DropletArgs D{};
        D.count = drops->count;
        for (int k = 0; k < drops->count; ++k) {
            D.x0[k] = drops->x0[k];
            D.y0[k] = drops->y0[k];
            D.r[k] = drops->radius[k];
        }
        D.mid = 0.5 * (p->rho_l + p->rho_v);
        D.half = 0.5 * (p->rho_l - p->rho_v);
        D.width = drops->width;
        D.jitter = drops->jitter;
        D.base = splitmix64_host(drops->seed);
        e = lbm::launch_droplets(c->kp, D, rho0, s);
        if (e != hipSuccess) { delete c; return create_fail(LBM_E_HIP, "create: droplets", e); }
    }
    if ((e = lbm::launch_init(c->kp, rho0, c->g[0], s)) != hipSuccess) { delete c; return create_fail(LBM_E_HIP, "create launch_init", e); }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { delete c; return create_fail(LBM_E_HIP, "create hipStreamSynchronize", e); }
    *out = c;
    return LBM_OK;
}

int lbm_create(const lbm_params* p, const double* gw_host, const double* rho0_host, void* d_ws,
               size_t ws_bytes, void* stream, lbm_ctx** out) {
    if (p && is_mask(p)) {
        if (out) *out = nullptr;
        return LBM_E_INVAL;  // a solid mask is given through lbm_create_masked
    }
    return create_impl(p, nullptr, gw_host, rho0_host, nullptr, d_ws, ws_bytes, stream, out);
}

int lbm_create_droplets(const lbm_params* p, const double* gw_host, const lbm_droplets* drops,
                        void* d_ws, size_t ws_bytes, void* stream, lbm_ctx** out) {
    if (p && is_mask(p)) {
        if (out) *out = nullptr;
        return LBM_E_INVAL;
    }
    if (!drops) {
        if (out) *out = nullptr;
        return LBM_E_INVAL;
    }
    return create_impl(p, nullptr, gw_host, nullptr, drops, d_ws, ws_bytes, stream, out);
}

int lbm_create_masked(const lbm_params* p, const uint8_t* solid_host, const double* gw_host,
                      const double* rho0_host, void* d_ws, size_t ws_bytes, void* stream,
                      lbm_ctx** out) {
    if (!p || !is_mask(p) || !solid_host || !gw_host) {
        if (out) *out = nullptr;
        return LBM_E_INVAL;
    }
    return create_impl(p, solid_host, gw_host, rho0_host, nullptr, d_ws, ws_bytes, stream, out);
}

int lbm_set_schedule(lbm_ctx* c, int32_t schedule) {
    if (!c) return LBM_E_INVAL;
    // 0 fused, 1 two-pass, 2 two steps per launch; 16 + t: fused with tile shape t;
    // 32 + t: two steps per launch with output tile t. A solid mask takes every schedule but
    // the overlapped fused tiles (16 + 4..7).
    if (c->kp.mask && schedule >= 20 && schedule < 32)
        return fail(c, LBM_E_INVAL, "a solid mask has no overlapped-tile schedule (tiles 4-7)");
    if (schedule >= 0 && schedule <= 2) { c->schedule = schedule; return LBM_OK; }
    if (schedule >= 16 && schedule < 16 + lbm::n_tiles()) {
        c->schedule = 0;
        c->tile = schedule - 16;
        return LBM_OK;
    }
    if (schedule >= 32 && schedule < 40) {
        c->schedule = 2;
        c->tile2 = schedule - 32;
        return LBM_OK;
    }
    return fail(c, LBM_E_INVAL, "unknown schedule");
}

// Launches of `n` steps of the context's schedule from buffer parity `cur`; *cur_out receives the
// parity holding the result (every launch swaps the buffers: two steps per launch make n/2 + n%2
// swaps, single steps n).
static hipError_t enqueue_steps(lbm_ctx* c, int64_t n, int cur, hipStream_t s, int* cur_out) {
    *cur_out = cur;
    if (c->schedule == 2) {
        for (; n >= 2; n -= 2) {
            hipError_t e = lbm::launch_step2(c->kp, c->tile2, c->g[cur], c->g[cur ^ 1], c->gw, s);
            if (e != hipSuccess) return e;
            cur ^= 1;
            *cur_out = cur;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        hipError_t e = lbm::launch_step(c->kp, c->schedule == 1 ? 1 : 0, c->tile, c->g[cur],
                                        c->g[cur ^ 1], c->psi, c->gw, s);
        if (e != hipSuccess) return e;
        cur ^= 1;
        *cur_out = cur;
    }
    return hipSuccess;
}

int lbm_step(lbm_ctx* c, int64_t n) {
    if (!c || n < 0) return LBM_E_INVAL;
    (void)hipGetLastError();  // report only errors of this call
    // direct launches: on this platform replaying captured graphs measured slower at every size
    int after = c->cur;
    hipError_t e = enqueue_steps(c, n, c->cur, c->stream, &after);
    if (e != hipSuccess) return hip_fail(c, e, "lbm_step");
    c->cur = after;
    c->step += n;
    return LBM_OK;
}

int64_t lbm_current_step(const lbm_ctx* c) { return c ? c->step : -1; }

// Observables record from the reduced sums of the observables kernel: density extremes,
// velocity maxima, mass, and the Kasa circle fit solved from its 3x3 normal equations.
// Height of the bottom wall plane: halfway between solid row 0 and fluid row 1 with bounce-back,
// on the boundary nodes of row 1 with the wet-node scheme (Sec. III.A).
static double wall_plane(int32_t walls) { return walls == LBM_WALLS_WET_NODE ? 1.0 : 0.5; }

static void obs_from_sums(const double* q, const lbm::ObsArgs& A, int64_t step, lbm_obs* out) {
    enum { O_MIN = 0, O_MAX, O_U, O_UL, O_MASS, O_BAD, O_N, O_SX, O_SY, O_SXX, O_SYY, O_SXY,
           O_SXR, O_SYR, O_SR };
    lbm_obs o{};
    o.step = step;
    o.rho_min = q[O_MIN];
    o.rho_max = q[O_MAX];
    o.umax = q[O_U];
    o.umax_liquid = q[O_UL] < 0 ? 0.0 : q[O_UL];
    o.mass = q[O_MASS];
    o.nonfinite = (int32_t)q[O_BAD];
    o.n_fit = (int32_t)q[O_N];
    o.theta_deg = o.xc = o.yc = o.r = NAN;
    if (o.n_fit >= 6) {
        // normal equations [Sxx Sxy Sx; Sxy Syy Sy; Sx Sy n] (D E F)^T = -(Sxr, Syr, Sr)^T
        double M[3][4] = {{q[O_SXX], q[O_SXY], q[O_SX], -q[O_SXR]},
                          {q[O_SXY], q[O_SYY], q[O_SY], -q[O_SYR]},
                          {q[O_SX], q[O_SY], q[O_N], -q[O_SR]}};
        for (int col = 0; col < 3; ++col) {  // Gaussian elimination, partial pivoting
            int piv = col;
            for (int r = col + 1; r < 3; ++r)
                if (std::fabs(M[r][col]) > std::fabs(M[piv][col])) piv = r;
            for (int k = 0; k < 4; ++k) std::swap(M[col][k], M[piv][k]);
            for (int r = 0; r < 3; ++r) {
                if (r == col || M[col][col] == 0.0) continue;
                double fct = M[r][col] / M[col][col];
                for (int k = col; k < 4; ++k) M[r][k] -= fct * M[col][k];
            }
        }
        const double D = M[0][3] / M[0][0], E = M[1][3] / M[1][1], F = M[2][3] / M[2][2];
        const double X = -D / 2.0, Y = -E / 2.0;
        const double r = std::sqrt(X * X + Y * Y - F);
        o.xc = X + A.cx;
        o.yc = Y + A.cy;
        o.r = r;
        const double cth = (A.cy - o.yc) / r;  // the shift origin is the wall plane
        if (std::isfinite(cth) && std::fabs(cth) <= 1.0) o.theta_deg = std::acos(cth) * 180.0 / M_PI;
    }
    *out = o;
}

int lbm_observables_plane(lbm_ctx* c, double x_lo, double x_hi, double y_wall, lbm_obs* out) {
    if (!c || !out || !std::isfinite(y_wall)) return LBM_E_INVAL;
    (void)hipGetLastError();  // report only errors of this call
    const KParams& P = c->kp;
    lbm::ObsArgs A;
    A.rho_mid = 0.5 * (c->p.rho_l + c->p.rho_v);
    A.y_min = y_wall + 3.0;
    A.x_lo = x_lo;
    A.x_hi = x_hi;
    A.cx = std::isfinite(x_lo) && std::isfinite(x_hi) ? 0.5 * (x_lo + x_hi) : 0.5 * P.nx;
    A.cy = y_wall;
    double* rho = c->g[c->cur ^ 1];  // the idle population buffer serves as scratch
    hipError_t e = lbm::launch_rho_psi(P, c->g[c->cur], c->psi, rho, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "observables psi");
    e = lbm::launch_obs(P, c->g[c->cur], rho, c->psi, c->gw, A, c->part, c->fin, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "observables");
    double q[32];
    e = host_copy(c->stream, q, c->fin, lbm::OBS_NQ * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "observables copy");

    obs_from_sums(q, A, c->step, out);
    return out->nonfinite ? LBM_E_NONFINITE : LBM_OK;
}

int lbm_observables_window(lbm_ctx* c, double x_lo, double x_hi, lbm_obs* out) {
    if (!c) return LBM_E_INVAL;
    return lbm_observables_plane(c, x_lo, x_hi, wall_plane(c->p.walls), out);
}

int lbm_record_contact_line(lbm_ctx* c, int64_t n, int32_t every, int32_t row, double* d_series,
                            size_t count) {
    if (!c || !d_series || n < 0 || every < 1 || n % every) return LBM_E_INVAL;
    if (row < c->kp.y_lo || row > c->kp.y_hi) return fail(c, LBM_E_INVAL, "row outside the fluid rows");
    const size_t samples = (size_t)(n / every) + 1;
    if (count < 2 * samples) return fail(c, LBM_E_SIZE, "series buffer too small");
    (void)hipGetLastError();  // report only errors of this call
    const double mid = 0.5 * (c->p.rho_l + c->p.rho_v);
    for (size_t k = 0; k < samples; ++k) {
        if (k) {
            int after = c->cur;
            hipError_t e = enqueue_steps(c, every, c->cur, c->stream, &after);
            if (e != hipSuccess) return hip_fail(c, e, "record steps");
            c->cur = after;
            c->step += every;
        }
        hipError_t e = lbm::launch_contact_line(c->kp, c->g[c->cur], row, mid, d_series + 2 * k,
                                                c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "contact line");
    }
    return LBM_OK;
}

int lbm_observables(lbm_ctx* c, lbm_obs* out) {
    return lbm_observables_window(c, -INFINITY, INFINITY, out);
}

int lbm_observables_of_state(const lbm_params* p, const double* d_f, const double* d_gw,
                             void* stream, lbm_obs* out) {
    if (!out || !d_f) return LBM_E_INVAL;
    std::string msg;
    int rc = validate(p, &msg);
    if (rc) {
        g_create_err = "observables_of_state: " + msg;
        return rc;
    }
    if (is_mask(p) || (p->walls && !d_gw) || ((uintptr_t)d_f) % 8 || ((uintptr_t)d_gw) % 8) {
        g_create_err = "observables_of_state: a solid mask, a missing G_w or a misaligned array";
        return LBM_E_INVAL;
    }
    // the caller's arrays are dense: row pitch nx, plane nx * ny
    Layout L{};
    L.pitch = p->nx;
    L.plane = (long long)p->nx * p->ny;
    const KParams P = kparams_of(p, L);
    const size_t plane_b = align_up((size_t)L.plane * sizeof(double), kAlign);
    const size_t part_b = align_up((size_t)lbm::obs_blocks(P) * lbm::OBS_NQ * sizeof(double), kAlign);
    const size_t need = 2 * plane_b + part_b + align_up(32 * sizeof(double), kAlign);
    if (need > kStaticScratchBytes) {
        g_create_err = "observables_of_state: the lattice needs " + std::to_string(need) +
                       " bytes of scratch, more than the " + std::to_string(kStaticScratchBytes) +
                       "-byte static array";
        return LBM_E_SIZE;
    }
    (void)hipGetLastError();  // report only errors of this call
    void* base = nullptr;
    hipError_t e = static_scratch(&base);
    if (e != hipSuccess) return create_fail(LBM_E_HIP, "observables_of_state: scratch address", e);
    char* w = (char*)base;
    double* rho = (double*)w;
    double* psi = (double*)(w + plane_b);
    double* part = (double*)(w + 2 * plane_b);
    double* fin = (double*)(w + 2 * plane_b + part_b);
    hipStream_t s = (hipStream_t)stream;
    // the array keeps the previous call's contents: rows no kernel below writes must read 0
    if (p->walls && !p->ghost_psi) {
        e = lbm::launch_zero(psi, (size_t)p->nx * sizeof(double), s);
        if (e == hipSuccess)
            e = lbm::launch_zero(psi + (size_t)(p->ny - 1) * p->nx, (size_t)p->nx * sizeof(double), s);
        if (e != hipSuccess) return create_fail(LBM_E_HIP, "observables_of_state: clear", e);
    }
    lbm::ObsArgs A;
    const double yw = wall_plane(p->walls);
    A.rho_mid = 0.5 * (p->rho_l + p->rho_v);
    A.y_min = yw + 3.0;
    A.x_lo = -INFINITY;
    A.x_hi = INFINITY;
    A.cx = 0.5 * P.nx;
    A.cy = yw;
    e = lbm::launch_rho_psi(P, d_f, psi, rho, s, true);
    if (e == hipSuccess) e = lbm::launch_obs(P, d_f, rho, psi, d_gw, A, part, fin, s, true);
    double q[32];
    if (e == hipSuccess) e = host_copy(s, q, fin, lbm::OBS_NQ * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return create_fail(LBM_E_HIP, "observables_of_state", e);
    obs_from_sums(q, A, 0, out);
    return out->nonfinite ? LBM_E_NONFINITE : LBM_OK;
}

// Read-outs use the idle population buffer as scratch: the next step overwrites it.
int lbm_read_rho(lbm_ctx* c, double* host, size_t count) {
    if (!c || !host) return LBM_E_INVAL;
    if (count < (size_t)c->p.nx * c->p.ny) return LBM_E_SIZE;
    const KParams& P = c->kp;
    double* scratch = c->g[c->cur ^ 1];
    hipError_t e = lbm::launch_zero(scratch, (size_t)P.plane * sizeof(double), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "read_rho memset");
    e = lbm::launch_rho_psi(P, c->g[c->cur], c->psi, scratch, c->stream);
    if (e == hipSuccess)
        e = download_field(c->stream, scratch, P.plane, P.pitch, 1, P.ny, P.nx, scratch + P.plane,
                           host);
    if (e != hipSuccess) return hip_fail(c, e, "read_rho");
    return LBM_OK;
}

int lbm_read_f(lbm_ctx* c, double* host, size_t count) {
    if (!c || !host) return LBM_E_INVAL;
    if (count < (size_t)9 * c->p.nx * c->p.ny) return LBM_E_SIZE;
    const KParams& P = c->kp;
    double* scratch = c->g[c->cur ^ 1];
    const size_t n = (size_t)9 * P.nx * P.ny;
    hipError_t e = lbm::launch_zero(scratch, n * sizeof(double), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "read_f memset");
    e = lbm::launch_pull(P, c->g[c->cur], scratch, c->stream, true);
    if (e == hipSuccess) e = host_copy(c->stream, host, scratch, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "read_f");
    return LBM_OK;
}

struct StateHeader {
    uint64_t magic;
    int64_t step;
    int32_t nx, ny;
    int32_t walls, pad;
};
static const uint64_t kMagic = 0x4C424D5354415445ULL;  // "LBMSTATE"

int lbm_state_size(const lbm_ctx* c, size_t* bytes) {
    if (!c || !bytes) return LBM_E_INVAL;
    *bytes = sizeof(StateHeader) + (size_t)9 * c->p.nx * c->p.ny * sizeof(double);
    return LBM_OK;
}

int lbm_save_state(lbm_ctx* c, void* host, size_t bytes) {
    size_t need;
    if (!c || !host) return LBM_E_INVAL;
    lbm_state_size(c, &need);
    if (bytes < need) return LBM_E_SIZE;
    StateHeader h{kMagic, c->step, c->p.nx, c->p.ny, c->p.walls, 0};
    std::memcpy(host, &h, sizeof h);
    const KParams& P = c->kp;
    hipError_t e = download_field(c->stream, c->g[c->cur], P.plane, P.pitch, 9, P.ny, P.nx,
                                  c->g[c->cur ^ 1], (double*)((char*)host + sizeof h));
    if (e != hipSuccess) return hip_fail(c, e, "save_state");
    return LBM_OK;
}

int lbm_load_state(lbm_ctx* c, const void* host, size_t bytes) {
    size_t need;
    if (!c || !host) return LBM_E_INVAL;
    lbm_state_size(c, &need);
    if (bytes < need) return LBM_E_SIZE;
    StateHeader h;
    std::memcpy(&h, host, sizeof h);
    if (h.magic != kMagic || h.nx != c->p.nx || h.ny != c->p.ny || h.walls != c->p.walls)
        return fail(c, LBM_E_STATE, "state blob does not match this context");
    const KParams& P = c->kp;
    const double* src = (const double*)((const char*)host + sizeof h);
    hipError_t e = upload_field(c->stream, src, 9, P.ny, P.nx, c->g[c->cur ^ 1], c->g[c->cur],
                                P.plane, P.pitch);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "load_state");
    c->step = h.step;
    return LBM_OK;
}

int lbm_set_gw(lbm_ctx* c, const double* gw_host) {
    if (!c || !gw_host) return LBM_E_INVAL;
    const int rows = c->kp.mask ? c->p.ny : 2;
    for (long long i = 0; i < (long long)rows * c->p.nx; ++i)
        if (!std::isfinite(gw_host[i])) return fail(c, LBM_E_INVAL, "non-finite G_w");
    hipError_t e = upload_field(c->stream, gw_host, 1, rows, c->p.nx, c->g[c->cur ^ 1], c->gw, 0,
                                c->kp.pitch);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_gw");
    return LBM_OK;
}


// ---- adjoint ------------------------------------------------------------------------------

int lbm_adjoint_workspace_size(const lbm_params* p, int64_t nsteps, int32_t K, size_t* bytes) {
    if (!bytes || nsteps < 1 || K < 1) return LBM_E_INVAL;
    int rc = validate(p, nullptr);
    if (rc) return rc;
    if (p->walls != LBM_WALLS_BOUNCE_BACK) return LBM_E_INVAL;  // objective and adjoint: bounce-back walls
    *bytes = adj_layout_of(p, nsteps, K, 2).total;
    return LBM_OK;
}

static int run_loss(lbm_ctx* c, double* sums) {
    hipError_t e = lbm::launch_loss(c->kp, c->g[c->cur], c->part, c->fin, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "loss");
    e = host_copy(c->stream, sums, c->fin, 3 * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "loss copy");
    return LBM_OK;
}

int lbm_loss(lbm_ctx* c, double w_centroid, double w_wet, double* L) {
    if (!c || !L || c->p.walls != LBM_WALLS_BOUNCE_BACK) return LBM_E_INVAL;
    double s[3];
    int rc = run_loss(c, s);
    if (rc) return rc;
    *L = w_centroid * s[1] / s[0] + w_wet * s[2];
    return std::isfinite(*L) ? LBM_OK : fail(c, LBM_E_NONFINITE, "non-finite loss");
}

// The auxiliary stream and events of lbm_backward, created on first use on the context's device.
static hipError_t adj_streams(lbm_ctx* c) {
    if (c->aux) return hipSuccess;
    hipError_t e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
    if (e != hipSuccess) {
        c->aux = nullptr;
        return e;
    }
    hipEvent_t* evs[5] = {&c->ev_start, &c->ev_rc[0], &c->ev_rc[1], &c->ev_free[0], &c->ev_free[1]};
    for (hipEvent_t* ev : evs)
        if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    return e;
}

int lbm_forward_ckpt(lbm_ctx* c, int64_t nsteps, int32_t K, void* d_adj, size_t bytes) {
    if (!c || !d_adj || nsteps < 1 || K < 1 || c->p.walls != LBM_WALLS_BOUNCE_BACK)
        return LBM_E_INVAL;
    AdjLayout A = adj_layout_of(&c->p, nsteps, K, 2);
    if (bytes < A.total) return fail(c, LBM_E_SIZE, "adjoint workspace too small");
    if (((uintptr_t)d_adj) % kAlign) return fail(c, LBM_E_INVAL, "adjoint workspace misaligned");
    char* w = (char*)d_adj;
    const size_t fb = (size_t)9 * c->kp.plane * sizeof(double);
    c->adj_start = c->step;
    c->adj_nsteps = nsteps;
    c->adj_K = K;
    c->adj_ws = d_adj;
    for (int64_t i = 0; i < nsteps; i += K) {
        hipError_t e = hipMemcpyAsync(w + A.off_ck + (size_t)(i / K) * A.fbytes, c->g[c->cur], fb,
                                      hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "checkpoint");
        int rc = lbm_step(c, std::min<int64_t>(K, nsteps - i));
        if (rc) return rc;
    }
    return LBM_OK;
}

int lbm_backward(lbm_ctx* c, int64_t nsteps, int32_t K, void* d_adj, size_t bytes,
                 double w_centroid, double w_wet, double* d_grad_gw) {
    if (!c || !d_adj || !d_grad_gw || nsteps < 1 || K < 1 || c->p.walls != LBM_WALLS_BOUNCE_BACK)
        return LBM_E_INVAL;
    AdjLayout A = adj_layout_of(&c->p, nsteps, K, 2);
    if (bytes < A.total) return fail(c, LBM_E_SIZE, "adjoint workspace too small");
    if (c->adj_ws != d_adj || c->adj_nsteps != nsteps || c->adj_K != K ||
        c->step != c->adj_start + nsteps)
        return fail(c, LBM_E_STATE, "backward does not follow the matching lbm_forward_ckpt");
    const KParams& P = c->kp;
    hipStream_t s = c->stream;
    char* w = (char*)d_adj;
    const size_t fb = (size_t)9 * P.plane * sizeof(double);
    (void)hipGetLastError();  // report only errors of this call
    hipError_t e = lbm::launch_zero(w + A.off_a, A.total - A.off_a, s);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint clear");

    double sums[3];
    int rc = run_loss(c, sums);
    if (rc) return rc;
    const double yc = sums[1] / sums[0];
    if (!std::isfinite(yc)) return fail(c, LBM_E_NONFINITE, "non-finite loss");
    double* a_buf[2] = {(double*)(w + A.off_a), (double*)(w + A.off_a + A.fbytes)};
    double* q_buf[2] = {(double*)(w + A.off_q), (double*)(w + A.off_q + 2 * A.pbytes)};
    double* p0_buf[2] = {(double*)(w + A.off_p0), (double*)(w + A.off_p0 + A.pbytes)};
    double* dpsi_buf[2] = {(double*)(w + A.off_dpsi), (double*)(w + A.off_dpsi + A.pbytes)};
    double* rv_buf[2] = {(double*)(w + A.off_rv), (double*)(w + A.off_rv + A.rbytes)};
    double* gg = (double*)(w + A.off_gg);
    e = lbm::launch_loss_seed(P, w_centroid, w_wet, yc, sums[0], p0_buf[0], dpsi_buf[0], s);
    if (e != hipSuccess) return hip_fail(c, e, "loss seed");
    // Segment j is recomputed from its checkpoint into store j % 2 on the auxiliary stream while
    // the context stream runs segment j + 1 in reverse; the reverse sweep of segment j waits for
    // its recomputation (ev_rc), and the recomputation of segment j - 2 into the same store waits
    // for the reverse sweep of segment j (ev_free).
    if ((e = adj_streams(c)) != hipSuccess) return hip_fail(c, e, "adjoint stream");
    auto seg = [&](int64_t j, int64_t i) {
        return (double*)(w + A.off_seg + ((size_t)(j & 1) * K + (size_t)i) * A.fbytes);
    };
    auto seg_len = [&](int64_t j) { return std::min<int64_t>(K, nsteps - j * K); };
    auto recompute = [&](int64_t j) -> hipError_t {
        hipStream_t a = c->aux;
        hipError_t r = hipMemcpyAsync(seg(j, 0), w + A.off_ck + (size_t)j * A.fbytes, fb,
                                      hipMemcpyDeviceToDevice, a);
        const int64_t len = seg_len(j);
        int64_t i = 0;
        // two steps per launch, the first one written too
        for (; i + 2 <= len - 1 && r == hipSuccess; i += 2)
            r = lbm::launch_step2(P, c->tile2, seg(j, i), seg(j, i + 2), c->gw, a, seg(j, i + 1));
        if (i + 1 <= len - 1 && r == hipSuccess)
            r = lbm::launch_step(P, 0, c->tile, seg(j, i), seg(j, i + 1), c->psi, c->gw, a);
        if (r == hipSuccess) r = hipEventRecord(c->ev_rc[j & 1], a);
        return r;
    };
    e = hipEventRecord(c->ev_start, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->aux, c->ev_start, 0);
    if (e == hipSuccess) e = recompute(A.nck - 1);
    if (e != hipSuccess) return hip_fail(c, e, "segment recompute");
    int k = 0;  // buffers of the later step
    for (int64_t j = A.nck - 1; j >= 0; --j) {
        if (j >= 1) {
            // the store of segment j - 1 last held segment j + 1
            if (j + 1 <= A.nck - 1) e = hipStreamWaitEvent(c->aux, c->ev_free[(j + 1) & 1], 0);
            if (e == hipSuccess) e = recompute(j - 1);
            if (e != hipSuccess) return hip_fail(c, e, "segment recompute");
        }
        e = hipStreamWaitEvent(s, c->ev_rc[j & 1], 0);
        if (e != hipSuccess) return hip_fail(c, e, "segment wait");
        // the segment's adjoint steps in reverse
        for (int64_t i = seg_len(j) - 1; i >= 0; --i) {
            lbm::AdjPtrs ap{seg(j, i),    a_buf[k],     q_buf[k],     p0_buf[k],
                            dpsi_buf[k],  rv_buf[k],    c->gw,        a_buf[k ^ 1],
                            q_buf[k ^ 1], p0_buf[k ^ 1], dpsi_buf[k ^ 1], rv_buf[k ^ 1], gg};
            e = lbm::launch_adj(P, ap, s);
            if (e != hipSuccess) return hip_fail(c, e, "adjoint step");
            k ^= 1;
        }
        e = hipEventRecord(c->ev_free[j & 1], s);
        if (e != hipSuccess) return hip_fail(c, e, "segment event");
    }
    e = lbm::launch_adj_gw(P, rv_buf[k], gg, s);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint wall gradient");
    e = lbm::launch_repack(gg, 0, P.pitch, d_grad_gw, 0, P.nx, P.nx, 2, 1, s);
    if (e != hipSuccess) return hip_fail(c, e, "gradient copy");
    return LBM_OK;
}


// ---- ensembles ------------------------------------------------------------------------------

struct lbm_batch {
    int32_t count;
    std::vector<lbm_params> p;
    std::vector<KParams> kp;
    std::vector<lbm::InstDesc> desc;  // host copy of the device table
    hipStream_t stream;
    char* ws;
    size_t bytes;
    lbm::InstDesc* d_inst;
    int* d_tile_inst;
    unsigned long long* d_bar;  // grid-barrier arrival counter of the persistent schedule
    int* d_flag;
    std::vector<double*> psi, part, fin;
    int ntiles;
    int cur;
    int64_t step;
    lbm_tune tune;
    int grid;  // persistent grid size
    int spin_limit;  // polls before a persistent grid barrier aborts the run
    int geo;   // lbm::GEO_ROWS, GEO_WET (some instance wet-node) or GEO_MASK (all masked)
    int eos;   // lbm::EOS_CS or EOS_PW shared by every instance, else EOS_ANY
    std::vector<int32_t> rows;  // contact-line rows of the last record call (host copy)
    int* d_rows;
    hipGraphExec_t graph[2];  // per-step schedule: kGraphChunk launches starting at parity 0 / 1
    hipGraphExec_t pgraph;    // persistent schedule: reset + persistent kernel for pgraph_n steps
    int64_t pgraph_n;
    int pgraph_cur;
    // last lbm_batch_forward_ckpt: where it started, its length and checkpoint interval
    int64_t adj_start, adj_nsteps;
    int32_t adj_K;
    const void* adj_ws;
    std::string err;
};

namespace {

constexpr int kGraphChunk = 64;


constexpr int kSpinLimit = 1 << 22;

// Polls a persistent grid barrier makes before it aborts the run: LBM_PERSISTENT_SPIN_LIMIT when
// set to a non-negative integer (read when an ensemble is created), else kSpinLimit.
static int spin_limit_from_env() {
    const char* v = std::getenv("LBM_PERSISTENT_SPIN_LIMIT");
    if (!v || !*v) return kSpinLimit;
    char* end = nullptr;
    const long n = std::strtol(v, &end, 10);
    if (*end != '\0' || n < 0 || n > (1L << 30)) return kSpinLimit;
    return (int)n;
}

struct BatchLayout {
    size_t off_desc, off_tiles, off_bar, off_rows, total;
    std::vector<size_t> off_inst;  // per instance: g0, g1, gw, psi, part, fin
    std::vector<Layout> L;
    int ntiles;
    std::vector<int> tile0, ntx, nty;
};

bool batch_layout(const lbm_params* p, int32_t count, int tile, BatchLayout* B) {
    int TX = 64, TY = 4;
    lbm::batch_tile_shape(tile, &TX, &TY);
    size_t o = 0;
    B->off_desc = o;
    o += align_up((size_t)count * sizeof(lbm::InstDesc), kAlign);
    long long nt = 0;
    B->tile0.resize(count); B->ntx.resize(count); B->nty.resize(count); B->L.resize(count);
    for (int i = 0; i < count; ++i) {
        const int ylo = y_lo_of(&p[i]), yhi = y_hi_of(&p[i]);
        B->ntx[i] = (p[i].nx + TX - 1) / TX;
        B->nty[i] = (yhi - ylo + TY) / TY;
        B->tile0[i] = (int)nt;
        nt += (long long)B->ntx[i] * B->nty[i];
        B->L[i] = layout_of(&p[i]);
    }
    if (nt > (1LL << 30)) return false;
    B->ntiles = (int)nt;
    B->off_tiles = o;
    o += align_up((size_t)nt * sizeof(int), kAlign);
    B->off_bar = o;  // the persistent schedule's control block
    o += align_up((size_t)lbm::kControlWords * 8, kAlign);
    B->off_rows = o;
    o += align_up((size_t)count * sizeof(int), kAlign);
    B->off_inst.resize(count);
    for (int i = 0; i < count; ++i) {
        B->off_inst[i] = o;
        o += B->L[i].total;
    }
    B->total = o;
    return true;
}

int batch_fail(lbm_batch* b, int code, const std::string& m) {
    if (b) b->err = m;
    return code;
}

int validate_tune(const lbm_tune* t) {
    if (!t) return LBM_OK;
    if (t->tile < 0 || t->tile > 4 || t->schedule < 0 || t->schedule > 2 || t->waves_per_cu < 0 ||
        t->reserved != 0)
        return LBM_E_INVAL;
    return LBM_OK;
}

}  // namespace

int lbm_batch_workspace_size(const lbm_params* p, int32_t count, const lbm_tune* tune,
                             size_t* bytes) {
    if (!p || count < 1 || !bytes) return LBM_E_INVAL;
    if (validate_tune(tune)) return LBM_E_INVAL;
    for (int i = 0; i < count; ++i) {
        int rc = validate(&p[i], nullptr);
        if (rc) return rc;
        if (is_mask(&p[i]) != is_mask(&p[0])) return LBM_E_INVAL;  // all masked or none
    }
    BatchLayout B;
    if (!batch_layout(p, count, tune ? tune->tile : 0, &B)) return LBM_E_INVAL;
    *bytes = B.total;
    return LBM_OK;
}

static int batch_create_impl(const lbm_params* p, int32_t count,
                             const uint8_t* const* solid_host, const double* const* gw_host,
                             const double* const* rho0_host, const lbm_tune* tune, void* d_ws,
                             size_t bytes, void* stream, lbm_batch** out) {
    if (!out) return LBM_E_INVAL;
    *out = nullptr;
    if (!p || count < 1 || !rho0_host || !gw_host || !d_ws) return LBM_E_INVAL;
    if (validate_tune(tune)) return LBM_E_INVAL;
    for (int i = 0; i < count; ++i) {
        int rc = validate(&p[i], nullptr);
        if (rc) return rc;
        // masked ensembles come with a mask for every instance, others with none
        if (is_mask(&p[i]) != (solid_host != nullptr)) return LBM_E_INVAL;
        if (solid_host && !solid_host[i]) return LBM_E_INVAL;
        if (!rho0_host[i] || (p[i].walls && !gw_host[i])) return LBM_E_INVAL;
    }
    lbm_tune tn = tune ? *tune : lbm_tune{1, 0, 0, 0};
    BatchLayout B;
    if (!batch_layout(p, count, tn.tile, &B)) return LBM_E_INVAL;
    if (bytes < B.total) return LBM_E_SIZE;
    if (((uintptr_t)d_ws) % kAlign) return LBM_E_INVAL;

    (void)hipGetLastError();  // report only errors of this call
    lbm_batch* b = new lbm_batch();
    b->count = count;
    b->p.assign(p, p + count);
    b->stream = (hipStream_t)stream;
    b->ws = (char*)d_ws;
    b->bytes = bytes;
    b->d_inst = (lbm::InstDesc*)(b->ws + B.off_desc);
    b->d_tile_inst = (int*)(b->ws + B.off_tiles);
    b->d_bar = (unsigned long long*)(b->ws + B.off_bar);
    b->d_flag = (int*)(b->ws + B.off_bar + 64);
    b->ntiles = B.ntiles;
    b->geo = solid_host ? lbm::GEO_MASK : lbm::GEO_ROWS;
    b->eos = p[0].eos == LBM_EOS_CS ? lbm::EOS_CS : lbm::EOS_PW;
    for (int i = 1; i < count; ++i)
        if (p[i].eos != p[0].eos) b->eos = lbm::EOS_ANY;
    for (int i = 0; i < count; ++i)
        if (p[i].walls == LBM_WALLS_WET_NODE) b->geo = lbm::GEO_WET;
    b->d_rows = (int*)(b->ws + B.off_rows);
    b->cur = 0;
    b->step = 0;
    b->tune = tn;
    b->graph[0] = b->graph[1] = nullptr;
    b->pgraph = nullptr;
    b->pgraph_n = -1;
    b->pgraph_cur = -1;
    b->adj_start = -1;
    b->adj_nsteps = 0;
    b->adj_K = 0;
    b->adj_ws = nullptr;
    hipStream_t s = b->stream;
    hipError_t e = lbm::launch_zero(b->ws, B.total, s);
    if (e != hipSuccess) { delete b; return create_fail(LBM_E_HIP, "create: workspace clear", e); }
    std::vector<int> tile_inst(B.ntiles);
    std::vector<std::vector<unsigned short>> links(count);  // host staging until the final sync
    for (int i = 0; i < count; ++i) {
        const Layout& L = B.L[i];
        char* base = b->ws + B.off_inst[i];
        KParams kp = kparams_of(&p[i], L);
        b->kp.push_back(kp);
        lbm::InstDesc d{};
        d.P = kp;
        d.g[0] = (double*)(base + L.off_g0);
        d.g[1] = (double*)(base + L.off_g1);
        d.gw = (double*)(base + L.off_gw);
        d.tile0 = B.tile0[i];
        d.ntx = B.ntx[i];
        d.nty = B.nty[i];
        b->desc.push_back(d);
        b->psi.push_back((double*)(base + L.off_psi));
        b->part.push_back((double*)(base + L.off_part));
        b->fin.push_back((double*)(base + L.off_fin));
        for (int t = 0; t < B.ntx[i] * B.nty[i]; ++t) tile_inst[B.tile0[i] + t] = i;
        const uint8_t* solid = solid_host ? solid_host[i] : nullptr;
        for (long long k = 0; k < (long long)p[i].nx * p[i].ny; ++k) {
            const int y = (int)(k / p[i].nx);
            if (solid ? solid[k] != 0 : (y < y_lo_of(&p[i]) || y > y_hi_of(&p[i]))) continue;
            if (!finite_pos(rho0_host[i][k]) || !psi_defined(&p[i], rho0_host[i][k])) { delete b; return LBM_E_INVAL; }
        }
        const int gw_rows = solid ? p[i].ny : 2;
        if (gw_host[i]) {
            for (long long k = 0; k < (long long)gw_rows * p[i].nx; ++k)
                if (!std::isfinite(gw_host[i][k])) { delete b; return LBM_E_INVAL; }
            e = upload_field(s, gw_host[i], 1, gw_rows, p[i].nx, d.g[1], d.gw, 0, L.pitch);
            if (e != hipSuccess) { delete b; return create_fail(LBM_E_HIP, "create: G_w copy", e); }
        }
        if (solid) {
            links[i] = mask_links(&p[i], solid, L.pitch);
            unsigned short* dl = (unsigned short*)(base + L.off_links);
            e = host_copy(s, dl, links[i].data(), links[i].size() * sizeof(unsigned short),
                          hipMemcpyHostToDevice);
            if (e != hipSuccess) { delete b; return create_fail(LBM_E_HIP, "create: links copy", e); }
            kp.links = dl;
            kp.gwn = d.gw;
            d.P = kp;
            b->kp.back() = kp;
            b->desc.back() = d;
        }
        double* rho0 = d.g[1] + L.plane;
        e = upload_field(s, rho0_host[i], 1, p[i].ny, p[i].nx, d.g[1], rho0, 0, L.pitch);
        if (e != hipSuccess) { delete b; return create_fail(LBM_E_HIP, "create: rho0 copy", e); }
        if ((e = lbm::launch_init(kp, rho0, d.g[0], s)) != hipSuccess) { delete b; return create_fail(LBM_E_HIP, "create launch_init", e); }
    }
    e = host_copy(s, b->d_inst, b->desc.data(), count * sizeof(lbm::InstDesc),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) { delete b; return create_fail(LBM_E_HIP, "create: descriptor copy", e); }
    e = host_copy(s, b->d_tile_inst, tile_inst.data(), B.ntiles * sizeof(int),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) { delete b; return create_fail(LBM_E_HIP, "create: tile table copy", e); }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { delete b; return create_fail(LBM_E_HIP, "create hipStreamSynchronize", e); }
    // persistent grid: co-resident workgroups only (occupancy x compute units)
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int occ = lbm::batch_persistent_occupancy(tn.tile);
    if (tn.waves_per_cu > 0 && tn.waves_per_cu < occ) occ = tn.waves_per_cu;
    b->grid = std::max(1, std::min(occ * cus, b->ntiles));
    b->spin_limit = spin_limit_from_env();
    *out = b;
    return LBM_OK;
}

int lbm_batch_create(const lbm_params* p, int32_t count, const double* const* gw_host,
                     const double* const* rho0_host, const lbm_tune* tune, void* d_ws,
                     size_t bytes, void* stream, lbm_batch** out) {
    if (p && count > 0 && is_mask(&p[0])) {
        if (out) *out = nullptr;
        return LBM_E_INVAL;  // masked ensembles: lbm_batch_create_masked
    }
    return batch_create_impl(p, count, nullptr, gw_host, rho0_host, tune, d_ws, bytes, stream,
                             out);
}

int lbm_batch_create_masked(const lbm_params* p, int32_t count, const uint8_t* const* solid_host,
                            const double* const* gw_host, const double* const* rho0_host,
                            const lbm_tune* tune, void* d_ws, size_t bytes, void* stream,
                            lbm_batch** out) {
    if (!solid_host) {
        if (out) *out = nullptr;
        return LBM_E_INVAL;
    }
    return batch_create_impl(p, count, solid_host, gw_host, rho0_host, tune, d_ws, bytes, stream,
                             out);
}

static int batch_direct(lbm_batch* b, int64_t n) {
    if (b->tune.schedule == 2) {
        for (; n >= 2; n -= 2) {
            hipError_t e = lbm::launch_batch_step2(b->tune.tile, b->geo, b->eos, b->d_inst,
                                                   b->d_tile_inst, b->ntiles, b->cur, b->stream);
            if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, std::string("batch step: ") + hipGetErrorString(e));
            b->cur ^= 1;
            b->step += 2;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        hipError_t e = lbm::launch_batch_step(b->tune.tile, b->geo, b->eos, b->d_inst, b->d_tile_inst,
                                              b->ntiles, b->cur, b->stream);
        if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, std::string("batch step: ") + hipGetErrorString(e));
        b->cur ^= 1;
        b->step += 1;
    }
    return LBM_OK;
}

// Captures `body` into an executable graph. The legacy default stream cannot be captured: there
// the caller launches directly (returns 1).
static int capture(lbm_batch* b, hipGraphExec_t* out, const std::function<hipError_t()>& body) {
    if (b->stream == nullptr) return 1;
    hipGraph_t g = nullptr;
    (void)hipGetLastError();
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    hipError_t e1 = body();
    e = hipStreamEndCapture(b->stream, &g);
    if (e1 != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return batch_fail(b, LBM_E_HIP, "capture");
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        *out = nullptr;
        (void)hipGetLastError();
        return 1;
    }
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int64_t n) {
    if (!b || n < 0) return LBM_E_INVAL;
    if (n == 0) return LBM_OK;
    (void)hipGetLastError();
    if (b->tune.schedule == 1) {
        // one launch of n / 2 two-step passes, and a per-step launch for an odd last step
        if (n > (int64_t)1 << 30) return batch_fail(b, LBM_E_INVAL, "too many steps in one call");
        const int cur = b->cur;
        const int npairs = (int)(n / 2);
        auto persistent = [&]() {
            hipError_t e = hipSuccess;
            if (npairs > 0)
                e = lbm::launch_batch_persistent(b->tune.tile, b->geo, b->eos, b->grid, b->d_inst,
                                                 b->d_tile_inst, b->ntiles, npairs, cur, b->d_bar,
                                                 b->d_flag, b->spin_limit, b->stream);
            if (e == hipSuccess && (n & 1))
                e = lbm::launch_batch_step(b->tune.tile, b->geo, b->eos, b->d_inst,
                                           b->d_tile_inst, b->ntiles, cur ^ (npairs & 1),
                                           b->stream);
            return e;
        };
        if (!b->pgraph || b->pgraph_n != n || b->pgraph_cur != cur) {
            if (b->pgraph) { (void)hipGraphExecDestroy(b->pgraph); b->pgraph = nullptr; }
            if (capture(b, &b->pgraph, persistent) == LBM_OK) {
                b->pgraph_n = n;
                b->pgraph_cur = cur;
            }
        }
        hipError_t e = b->pgraph ? hipGraphLaunch(b->pgraph, b->stream) : persistent();
        if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "persistent launch");
        b->cur ^= (npairs & 1) ^ (int)(n & 1);
        b->step += n;
        return LBM_OK;
    }
    // per-step schedule: replay a graph of kGraphChunk launches, then the remainder directly
    int64_t chunks = n / kGraphChunk;
    for (int64_t k = 0; k < chunks; ++k) {
        const int cur = b->cur;
        if (!b->graph[cur]) {
            int rc = capture(b, &b->graph[cur], [&]() {
                const bool two = b->tune.schedule == 2;  // two steps per launch
                for (int i = 0; i < (two ? kGraphChunk / 2 : kGraphChunk); ++i) {
                    hipError_t e = two ? lbm::launch_batch_step2(b->tune.tile, b->geo, b->eos, b->d_inst,
                                                                 b->d_tile_inst, b->ntiles,
                                                                 (cur + i) & 1, b->stream)
                                       : lbm::launch_batch_step(b->tune.tile, b->geo, b->eos, b->d_inst,
                                                                b->d_tile_inst, b->ntiles,
                                                                (cur + i) & 1, b->stream);
                    if (e != hipSuccess) return e;
                }
                return hipSuccess;
            });
            if (rc != LBM_OK) return batch_direct(b, n - k * kGraphChunk);  // no graph here
        }
        hipError_t e = hipGraphLaunch(b->graph[cur], b->stream);
        if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "graph launch");
        b->step += kGraphChunk;  // an even number of buffer swaps: parity unchanged
    }
    return batch_direct(b, n - chunks * kGraphChunk);
}

static int batch_check_abort(lbm_batch* b) {
    int flag = 0;
    hipError_t e = host_copy(b->stream, &flag, b->d_flag, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "flag read");
    if (flag) return batch_fail(b, LBM_E_HIP, "grid barrier timed out: workgroups not co-resident");
    return LBM_OK;
}

int lbm_batch_observables_plane(lbm_batch* b, const double* y_wall, lbm_obs* out) {
    if (!b || !out) return LBM_E_INVAL;
    if (y_wall)
        for (int i = 0; i < b->count; ++i)
            if (!std::isfinite(y_wall[i])) return LBM_E_INVAL;
    int rc = batch_check_abort(b);
    if (rc) return rc;
    std::vector<double> q((size_t)b->count * 32);
    std::vector<lbm::ObsArgs> args(b->count);
    for (int i = 0; i < b->count; ++i) {
        const KParams& P = b->kp[i];
        const lbm::InstDesc& d = b->desc[i];
        lbm::ObsArgs& A = args[i];
        const double yw = y_wall ? y_wall[i] : wall_plane(b->p[i].walls);
        A.rho_mid = 0.5 * (b->p[i].rho_l + b->p[i].rho_v);
        A.y_min = yw + 3.0;
        A.x_lo = -INFINITY;
        A.x_hi = INFINITY;
        A.cx = 0.5 * P.nx;
        A.cy = yw;
        double* rho = d.g[b->cur ^ 1];
        hipError_t e = lbm::launch_rho_psi(P, d.g[b->cur], b->psi[i], rho, b->stream);
        if (e == hipSuccess)
            e = lbm::launch_obs(P, d.g[b->cur], rho, b->psi[i], d.gw, A, b->part[i], b->fin[i],
                                b->stream);
        if (e == hipSuccess)
            e = host_copy(b->stream, q.data() + (size_t)i * 32, b->fin[i],
                          lbm::OBS_NQ * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "batch observables");
    }
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "batch observables sync");
    int bad = 0;
    for (int i = 0; i < b->count; ++i) {
        obs_from_sums(q.data() + (size_t)i * 32, args[i], b->step, &out[i]);
        bad |= out[i].nonfinite != 0;
    }
    return bad ? LBM_E_NONFINITE : LBM_OK;
}

int lbm_batch_observables(lbm_batch* b, lbm_obs* out) {
    return lbm_batch_observables_plane(b, nullptr, out);
}

int lbm_batch_record_contact_line(lbm_batch* b, int64_t n, int32_t every, const int32_t* rows,
                                  double* d_series, size_t count) {
    if (!b || !rows || !d_series || n < 0 || every < 1 || n % every) return LBM_E_INVAL;
    for (int i = 0; i < b->count; ++i)
        if (rows[i] < b->kp[i].y_lo || rows[i] > b->kp[i].y_hi)
            return batch_fail(b, LBM_E_INVAL, "row outside the fluid rows");
    const size_t samples = (size_t)(n / every) + 1;
    if (count < 2 * samples * (size_t)b->count) return batch_fail(b, LBM_E_SIZE, "series buffer too small");
    int rc = batch_check_abort(b);
    if (rc) return rc;
    (void)hipGetLastError();
    b->rows.assign(rows, rows + b->count);  // kept alive for the asynchronous copy
    hipError_t e = host_copy(b->stream, b->d_rows, b->rows.data(), b->count * sizeof(int),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "record rows");
    for (size_t k = 0; k < samples; ++k) {
        if (k) {
            rc = lbm_batch_step(b, every);
            if (rc) return rc;
        }
        e = lbm::launch_batch_contact_line(b->d_inst, b->d_rows, b->count, b->cur,
                                           d_series + 2 * (size_t)b->count * k, b->stream);
        if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "batch contact line");
    }
    return LBM_OK;
}

int lbm_batch_read_f(lbm_batch* b, int32_t index, double* host, size_t count) {
    if (!b || !host || index < 0 || index >= b->count) return LBM_E_INVAL;
    int rc = batch_check_abort(b);
    if (rc) return rc;
    const KParams& P = b->kp[index];
    if (count < (size_t)9 * P.nx * P.ny) return LBM_E_SIZE;
    const lbm::InstDesc& d = b->desc[index];
    double* scratch = d.g[b->cur ^ 1];  // the idle buffer: the next step overwrites it
    const size_t n = (size_t)9 * P.nx * P.ny;
    hipError_t e = lbm::launch_zero(scratch, n * sizeof(double), b->stream);
    if (e == hipSuccess) e = lbm::launch_pull(P, d.g[b->cur], scratch, b->stream, true);
    if (e == hipSuccess) e = host_copy(b->stream, host, scratch, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "batch read");
    return LBM_OK;
}


int lbm_batch_save_state(lbm_batch* b, int32_t index, void* host, size_t bytes) {
    if (!b || !host || index < 0 || index >= b->count) return LBM_E_INVAL;
    int rc = batch_check_abort(b);
    if (rc) return rc;
    const KParams& P = b->kp[index];
    const size_t need = sizeof(StateHeader) + (size_t)9 * P.nx * P.ny * sizeof(double);
    if (bytes < need) return LBM_E_SIZE;
    StateHeader h{kMagic, b->step, P.nx, P.ny, P.walls, 0};
    std::memcpy(host, &h, sizeof h);
    double* dst = (double*)((char*)host + sizeof h);
    const lbm::InstDesc& d = b->desc[index];
    hipError_t e = download_field(b->stream, d.g[b->cur], P.plane, P.pitch, 9, P.ny, P.nx,
                                  d.g[b->cur ^ 1], dst);
    if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "batch save state");
    return LBM_OK;
}

int64_t lbm_batch_current_step(const lbm_batch* b) { return b ? b->step : -1; }

int lbm_batch_get_tune(const lbm_batch* b, lbm_tune* t, int32_t* grid) {
    if (!b || !t) return LBM_E_INVAL;
    *t = b->tune;
    if (grid) *grid = b->grid;
    return LBM_OK;
}

// ---- ensemble adjoint --------------------------------------------------------------------------

namespace {

// Adjoint workspace of an ensemble: the instance table and the work-lists of 64 x 4 tiles (reverse
// steps) and 64 x 8 tiles (two-step recomputation), then per
// instance the single-lattice adjoint layout (checkpoints, segment, adjoint buffers, gradient).
struct BatchAdjLayout {
    size_t off_inst, off_tiles, off_tiles8, total;
    std::vector<size_t> off;
    std::vector<AdjLayout> A;
    std::vector<int> tile0, ntx, nty, tile0_8, nty8;
    int ntiles, ntiles8;  // 64 x 4 (reverse steps) and 64 x 8 (two-step recomputation) tiles
};

int batch_adj_layout(const lbm_batch* b, int64_t nsteps, int32_t K, BatchAdjLayout* L) {
    if (nsteps < 1 || K < 1) return LBM_E_INVAL;
    for (int i = 0; i < b->count; ++i)
        if (b->p[i].walls != LBM_WALLS_BOUNCE_BACK) return LBM_E_INVAL;
    size_t o = 0;
    L->off_inst = o;
    o += align_up((size_t)b->count * sizeof(lbm::AdjInst), kAlign);
    long long nt = 0, nt8 = 0;
    L->tile0.resize(b->count); L->ntx.resize(b->count); L->nty.resize(b->count);
    L->tile0_8.resize(b->count); L->nty8.resize(b->count);
    L->A.resize(b->count); L->off.resize(b->count);
    for (int i = 0; i < b->count; ++i) {
        const KParams& P = b->kp[i];
        L->ntx[i] = (P.nx + 63) / 64;
        L->nty[i] = (P.y_hi - P.y_lo + 4) / 4;
        L->nty8[i] = (P.y_hi - P.y_lo + 8) / 8;
        L->tile0[i] = (int)nt;
        L->tile0_8[i] = (int)nt8;
        nt += (long long)L->ntx[i] * L->nty[i];
        nt8 += (long long)L->ntx[i] * L->nty8[i];
    }
    if (nt > (1LL << 30)) return LBM_E_INVAL;
    L->ntiles = (int)nt;
    L->ntiles8 = (int)nt8;
    L->off_tiles = o;
    o += align_up((size_t)nt * sizeof(int), kAlign);
    L->off_tiles8 = o;
    o += align_up((size_t)nt8 * sizeof(int), kAlign);
    for (int i = 0; i < b->count; ++i) {
        L->A[i] = adj_layout_of(&b->p[i], nsteps, K, 1);
        L->off[i] = o;
        o += L->A[i].total;
    }
    L->total = o;
    return LBM_OK;
}

}  // namespace

int lbm_batch_adjoint_workspace_size(const lbm_batch* b, int64_t nsteps, int32_t K,
                                     size_t* bytes) {
    if (!b || !bytes) return LBM_E_INVAL;
    BatchAdjLayout L;
    int rc = batch_adj_layout(b, nsteps, K, &L);
    if (rc) return rc;
    *bytes = L.total;
    return LBM_OK;
}

int lbm_batch_forward_ckpt(lbm_batch* b, int64_t nsteps, int32_t K, void* d_adj, size_t bytes) {
    if (!b || !d_adj) return LBM_E_INVAL;
    BatchAdjLayout L;
    int rc = batch_adj_layout(b, nsteps, K, &L);
    if (rc) return batch_fail(b, rc, "ensemble adjoint: bounce-back walls only, nsteps, K >= 1");
    if (bytes < L.total) return batch_fail(b, LBM_E_SIZE, "adjoint workspace too small");
    if (((uintptr_t)d_adj) % kAlign) return batch_fail(b, LBM_E_INVAL, "adjoint workspace misaligned");
    (void)hipGetLastError();
    char* w = (char*)d_adj;
    b->adj_start = b->step;
    b->adj_nsteps = nsteps;
    b->adj_K = K;
    b->adj_ws = d_adj;
    for (int64_t i = 0; i < nsteps; i += K) {
        for (int k = 0; k < b->count; ++k) {
            const size_t fb = (size_t)9 * b->kp[k].plane * sizeof(double);
            hipError_t e = hipMemcpyAsync(w + L.off[k] + L.A[k].off_ck + (size_t)(i / K) * L.A[k].fbytes,
                                          b->desc[k].g[b->cur], fb, hipMemcpyDeviceToDevice,
                                          b->stream);
            if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "checkpoint");
        }
        rc = lbm_batch_step(b, std::min<int64_t>(K, nsteps - i));
        if (rc) return rc;
    }
    return LBM_OK;
}

// Loss sums (sum phi, sum phi (y - 1/2), sum_x phi(x, 1)) of instance i's current state.
static int batch_loss_sums(lbm_batch* b, int i, double* sums) {
    hipError_t e = lbm::launch_loss(b->kp[i], b->desc[i].g[b->cur], b->part[i], b->fin[i],
                                    b->stream);
    if (e == hipSuccess) e = host_copy(b->stream, sums, b->fin[i], 3 * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "ensemble loss");
    return LBM_OK;
}

int lbm_batch_loss(lbm_batch* b, double w_centroid, double w_wet, double* L) {
    if (!b || !L) return LBM_E_INVAL;
    for (int i = 0; i < b->count; ++i)
        if (b->p[i].walls != LBM_WALLS_BOUNCE_BACK) return LBM_E_INVAL;
    int rc = batch_check_abort(b);
    if (rc) return rc;
    int bad = 0;
    for (int i = 0; i < b->count; ++i) {
        double s[3];
        if ((rc = batch_loss_sums(b, i, s))) return rc;
        L[i] = w_centroid * s[1] / s[0] + w_wet * s[2];
        bad |= !std::isfinite(L[i]);
    }
    return bad ? batch_fail(b, LBM_E_NONFINITE, "non-finite loss") : LBM_OK;
}

int lbm_batch_backward(lbm_batch* b, int64_t nsteps, int32_t K, void* d_adj, size_t bytes,
                       double w_centroid, double w_wet, double* d_grad_gw) {
    if (!b || !d_adj || !d_grad_gw) return LBM_E_INVAL;
    BatchAdjLayout L;
    int rc = batch_adj_layout(b, nsteps, K, &L);
    if (rc) return batch_fail(b, rc, "ensemble adjoint: bounce-back walls only, nsteps, K >= 1");
    if (bytes < L.total) return batch_fail(b, LBM_E_SIZE, "adjoint workspace too small");
    if (b->adj_ws != d_adj || b->adj_nsteps != nsteps || b->adj_K != K ||
        b->step != b->adj_start + nsteps)
        return batch_fail(b, LBM_E_STATE, "backward does not follow the matching forward_ckpt");
    if ((rc = batch_check_abort(b))) return rc;
    (void)hipGetLastError();
    hipStream_t s = b->stream;
    char* w = (char*)d_adj;
    // instance table and work-list
    std::vector<lbm::AdjInst> inst(b->count);
    std::vector<int> tile_inst(L.ntiles), tile_inst8(L.ntiles8);
    int max_nx = 0;
    for (int i = 0; i < b->count; ++i) {
        const AdjLayout& A = L.A[i];
        char* base = w + L.off[i];
        lbm::AdjInst& d = inst[i];
        d = lbm::AdjInst{};
        d.P = b->kp[i];
        d.seg = (double*)(base + A.off_seg);
        d.fstride = (long long)(A.fbytes / sizeof(double));
        for (int k = 0; k < 2; ++k) {
            d.a[k] = (double*)(base + A.off_a + k * A.fbytes);
            d.q[k] = (double*)(base + A.off_q + 2 * k * A.pbytes);
            d.p0[k] = (double*)(base + A.off_p0 + k * A.pbytes);
            d.dpsi[k] = (double*)(base + A.off_dpsi + k * A.pbytes);
            d.rv[k] = (double*)(base + A.off_rv + k * A.rbytes);
        }
        d.gw = b->desc[i].gw;
        d.gg = (double*)(base + A.off_gg);
        d.tile0 = L.tile0[i];
        d.ntx = L.ntx[i];
        d.nty = L.nty[i];
        d.tile0_8 = L.tile0_8[i];
        d.nty8 = L.nty8[i];
        for (int t = 0; t < L.ntx[i] * L.nty[i]; ++t) tile_inst[L.tile0[i] + t] = i;
        for (int t = 0; t < L.ntx[i] * L.nty8[i]; ++t) tile_inst8[L.tile0_8[i] + t] = i;
        max_nx = std::max(max_nx, d.P.nx);
        hipError_t e = lbm::launch_zero(base + A.off_a, A.total - A.off_a, s);
        if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "adjoint clear");
    }
    lbm::AdjInst* d_inst = (lbm::AdjInst*)(w + L.off_inst);
    int* d_tiles = (int*)(w + L.off_tiles);
    int* d_tiles8 = (int*)(w + L.off_tiles8);
    hipError_t e = host_copy(s, d_inst, inst.data(), inst.size() * sizeof(lbm::AdjInst),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = host_copy(s, d_tiles, tile_inst.data(), tile_inst.size() * sizeof(int),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = host_copy(s, d_tiles8, tile_inst8.data(), tile_inst8.size() * sizeof(int),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "adjoint tables");
    // the objective of every instance seeds its adjoint
    for (int i = 0; i < b->count; ++i) {
        double sums[3];
        if ((rc = batch_loss_sums(b, i, sums))) return rc;
        const double yc = sums[1] / sums[0];
        if (!std::isfinite(yc)) return batch_fail(b, LBM_E_NONFINITE, "non-finite loss");
        e = lbm::launch_loss_seed(b->kp[i], w_centroid, w_wet, yc, sums[0], inst[i].p0[0],
                                  inst[i].dpsi[0], s);
        if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "loss seed");
    }
    const int64_t nck = (nsteps + K - 1) / K;
    int k = 0;  // buffers of the later step
    for (int64_t j = nck - 1; j >= 0; --j) {
        const int64_t len = std::min<int64_t>(K, nsteps - j * K);
        for (int i = 0; i < b->count && e == hipSuccess; ++i)
            e = hipMemcpyAsync(inst[i].seg, w + L.off[i] + L.A[i].off_ck + (size_t)j * L.A[i].fbytes,
                               (size_t)9 * b->kp[i].plane * sizeof(double), hipMemcpyDeviceToDevice, s);
        int64_t i = 0;
        for (; i + 2 <= len - 1 && e == hipSuccess; i += 2)
            e = lbm::launch_batch_seg_step2(b->eos, d_inst, d_tiles8, L.ntiles8, (int)i, s);
        if (i + 1 <= len - 1 && e == hipSuccess)
            e = lbm::launch_batch_seg_step(b->eos, d_inst, d_tiles, L.ntiles, (int)i, s);
        for (i = len - 1; i >= 0 && e == hipSuccess; --i) {
            e = lbm::launch_batch_adj(b->eos, d_inst, d_tiles, L.ntiles, (int)i, k, s);
            k ^= 1;
        }
        if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "ensemble adjoint segment");
    }
    e = lbm::launch_batch_adj_gw(d_inst, b->count, max_nx, k, s);
    size_t off = 0;
    for (int i = 0; i < b->count && e == hipSuccess; ++i) {
        const KParams& P = b->kp[i];
        e = lbm::launch_repack(inst[i].gg, 0, P.pitch, d_grad_gw + off, 0, P.nx, P.nx, 2, 1, s);
        off += (size_t)2 * P.nx;
    }
    if (e != hipSuccess) return batch_fail(b, LBM_E_HIP, "ensemble adjoint gradient");
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* b) {
    if (!b) return LBM_E_INVAL;
    // queued launches (graph replays among them) still read and write the workspace: let them
    // finish before the graphs go and the caller may release the workspace
    const hipError_t e = hipStreamSynchronize(b->stream);
    for (auto& g : b->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (b->pgraph) (void)hipGraphExecDestroy(b->pgraph);
    delete b;
    return e == hipSuccess ? LBM_OK : LBM_E_HIP;
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : g_create_err.c_str(); }

// Try every tile shape x schedule (and, for the persistent schedule, the full and half
// occupancy) on the given ensemble for `steps` steps each; return the fastest in *best and its
// time in *ms. The workspace must hold lbm_batch_workspace_size(p, count, NULL) bytes.
int lbm_autotune(const lbm_params* p, int32_t count, const double* const* gw_host,
                 const double* const* rho0_host, void* d_ws, size_t bytes, void* stream,
                 int32_t steps, lbm_tune* best, double* best_ms) {
    if (!best || steps < 1) return LBM_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LBM_E_HIP;
    double best_t = INFINITY;
    int rc_all = LBM_E_INVAL;
    // two sweeps over the candidates: the first also brings the device to its working clocks,
    // and each candidate counts with its faster run
    for (int sweep = 0; sweep < 2; ++sweep) {
        for (int tile = 0; tile < 5; ++tile) {
            for (int sched = 0; sched < 3; ++sched) {
                for (int half = 0; half < (sched == 1 ? 2 : 1); ++half) {
                    lbm_tune t{tile, 0, 0, sched};
                    size_t need;
                    if (lbm_batch_workspace_size(p, count, &t, &need) || need > bytes) continue;
                    if (half) {
                        int occ = lbm::batch_persistent_occupancy(tile);
                        if (occ < 2) continue;
                        t.waves_per_cu = occ / 2;
                    }
                    lbm_batch* b = nullptr;
                    if (lbm_batch_create(p, count, gw_host, rho0_host, &t, d_ws, bytes, stream,
                                         &b))
                        continue;
                    // warm-up (captures graphs), then the timed step count once: its graph is
                    // reused by the timed run
                    int rc = lbm_batch_step(b, 2);
                    if (!rc) rc = lbm_batch_step(b, steps);
                    (void)hipStreamSynchronize(s);
                    (void)hipEventRecord(e0, s);
                    if (!rc) rc = lbm_batch_step(b, steps);
                    (void)hipEventRecord(e1, s);
                    (void)hipEventSynchronize(e1);
                    if (!rc) rc = batch_check_abort(b);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    lbm_batch_destroy(b);
                    if (rc) continue;
                    rc_all = LBM_OK;
                    if (ms < best_t) {
                        best_t = ms;
                        *best = t;
                    }
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_ms) *best_ms = best_t;
    return rc_all;
}

int lbm_fp64_probe(const double* d_a, const double* d_b, double* d_sqrt, double* d_quot,
                   size_t n, void* stream) {
    if (n == 0) return LBM_OK;
    // at most 2^36 elements: 2^28 workgroups of 256, within the grid's x limit
    if (!d_a || !d_b || !d_sqrt || !d_quot || n > ((size_t)1 << 36)) return LBM_E_INVAL;
    (void)hipGetLastError();
    const hipError_t e = lbm::launch_fp64_probe(d_a, d_b, d_sqrt, d_quot, (long long)n,
                                                (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : create_fail(LBM_E_HIP, "fp64 probe", e);
}

int lbm_destroy(lbm_ctx* c) {
    if (!c) return LBM_E_INVAL;
    // queued launches still use the workspace: the caller may release it once this returns
    hipError_t e = hipStreamSynchronize(c->stream);
    if (c->aux) {
        const hipError_t e2 = hipStreamSynchronize(c->aux);
        if (e == hipSuccess) e = e2;
        for (hipEvent_t ev : {c->ev_start, c->ev_rc[0], c->ev_rc[1], c->ev_free[0], c->ev_free[1]})
            if (ev) (void)hipEventDestroy(ev);
        (void)hipStreamDestroy(c->aux);
    }
    delete c;
    return e == hipSuccess ? LBM_OK : LBM_E_HIP;
}

}  // extern "C"
