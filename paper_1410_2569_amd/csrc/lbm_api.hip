// lbm_api.hip -- C ABI of liblbm (declared in include/lbm.h): parameter validation, workspace
// carving, stream-ordered launches of the kernels in lbm_kernels.hip, observables post-processing
// and the Carnahan-Starling Maxwell construction.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

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
    std::string err;
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    int pitch;
    long long plane;  // doubles
    size_t off_g0, off_g1, off_psi, off_gw, off_part, off_fin, total;
};

Layout layout_of(const lbm_params* p) {
    Layout L;
    L.pitch = (int)align_up((size_t)p->nx, 32);
    L.plane = (long long)p->ny * L.pitch;
    size_t fbytes = align_up((size_t)(9 * L.plane) * sizeof(double), kAlign);
    size_t o = 0;
    L.off_g0 = o; o += fbytes;
    L.off_g1 = o; o += fbytes;
    L.off_psi = o; o += align_up((size_t)L.plane * sizeof(double), kAlign);
    L.off_gw = o; o += align_up((size_t)2 * L.pitch * sizeof(double), kAlign);
    KParams tmp{};
    tmp.nx = p->nx; tmp.ny = p->ny;
    tmp.y_lo = p->walls ? 1 : 0; tmp.y_hi = p->walls ? p->ny - 2 : p->ny - 1;
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
    if (p->walls != 0 && p->walls != 1) return bad("walls must be 0 or 1");
    if (p->ghost_psi != 0 && p->ghost_psi != 1) return bad("ghost_psi must be 0 or 1");
    if (p->nx < 3) return bad("nx must be >= 3");
    if (p->ny < (p->walls ? 4 : 3)) return bad("ny must be >= 4 with walls (>= 3 without)");
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
    k.y_lo = p->walls ? 1 : 0;
    k.y_hi = p->walls ? p->ny - 2 : p->ny - 1;
    k.RT = p->R * p->T; k.a = p->a; k.b4 = p->b / 4.0;
    k.rho1 = p->rho1; k.rho2 = p->rho2; k.th_v = p->th_v; k.th_m = p->th_m; k.th_l = p->th_l;
    k.p1 = p->rho1 * p->th_v;
    k.p2 = k.p1 + (p->rho2 - p->rho1) * p->th_m;
    k.two_over_G = 2.0 / p->G;
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

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : ""; }

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

int lbm_workspace_size(const lbm_params* p, size_t* bytes) {
    if (!bytes) return LBM_E_INVAL;
    int rc = validate(p, nullptr);
    if (rc) return rc;
    *bytes = layout_of(p).total;
    return LBM_OK;
}

int lbm_create(const lbm_params* p, const double* gw_host, const double* rho0_host, void* d_ws,
               size_t ws_bytes, void* stream, lbm_ctx** out) {
    if (!out) return LBM_E_INVAL;
    *out = nullptr;
    std::string msg;
    int rc = validate(p, &msg);
    if (rc) return rc;
    if (!rho0_host || !d_ws) return LBM_E_INVAL;
    if (p->walls && !gw_host) return LBM_E_INVAL;
    for (long long i = 0; i < (long long)p->nx * p->ny; ++i) {
        const int y = (int)(i / p->nx);
        if (p->walls && (y == 0 || y == p->ny - 1)) continue;
        if (!finite_pos(rho0_host[i])) return LBM_E_INVAL;
    }
    if (gw_host)
        for (int i = 0; i < 2 * p->nx; ++i)
            if (!std::isfinite(gw_host[i])) return LBM_E_INVAL;
    Layout L = layout_of(p);
    if (ws_bytes < L.total) return LBM_E_SIZE;
    if (((uintptr_t)d_ws) % kAlign) return LBM_E_INVAL;

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
    c->schedule = 0;
    c->tile = 1;

    hipStream_t s = c->stream;
    hipError_t e;
    if ((e = hipMemsetAsync(c->ws, 0, L.total, s)) != hipSuccess) { delete c; return LBM_E_HIP; }
    if (gw_host) {
        e = hipMemcpy2DAsync(c->gw, L.pitch * sizeof(double), gw_host, p->nx * sizeof(double),
                             p->nx * sizeof(double), 2, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) { delete c; return LBM_E_HIP; }
    }
    // stage rho0 in the second population buffer, then build the first from it
    e = hipMemcpy2DAsync(c->g[1], L.pitch * sizeof(double), rho0_host, p->nx * sizeof(double),
                         p->nx * sizeof(double), p->ny, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) { delete c; return LBM_E_HIP; }
    if ((e = lbm::launch_init(c->kp, c->g[1], c->g[0], s)) != hipSuccess) { delete c; return LBM_E_HIP; }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { delete c; return LBM_E_HIP; }
    *out = c;
    return LBM_OK;
}

int lbm_set_schedule(lbm_ctx* c, int32_t schedule) {
    if (!c) return LBM_E_INVAL;
    // schedule: 0 fused (tile = default), 1 two-pass; 16 + t: fused with tile shape t
    if (schedule == 0 || schedule == 1) { c->schedule = schedule; return LBM_OK; }
    if (schedule >= 16 && schedule < 16 + lbm::n_tiles()) {
        c->schedule = 0;
        c->tile = schedule - 16;
        return LBM_OK;
    }
    return fail(c, LBM_E_INVAL, "unknown schedule");
}

int lbm_step(lbm_ctx* c, int64_t n) {
    if (!c || n < 0) return LBM_E_INVAL;
    for (int64_t i = 0; i < n; ++i) {
        hipError_t e = lbm::launch_step(c->kp, c->schedule, c->tile, c->g[c->cur],
                                        c->g[c->cur ^ 1], c->psi, c->gw, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "lbm_step");
        c->cur ^= 1;
        c->step += 1;
    }
    return LBM_OK;
}

int64_t lbm_current_step(const lbm_ctx* c) { return c ? c->step : -1; }

int lbm_observables_window(lbm_ctx* c, double x_lo, double x_hi, lbm_obs* out) {
    if (!c || !out) return LBM_E_INVAL;
    const KParams& P = c->kp;
    lbm::ObsArgs A;
    A.rho_mid = 0.5 * (c->p.rho_l + c->p.rho_v);
    A.y_min = 0.5 + 3.0;
    A.x_lo = x_lo;
    A.x_hi = x_hi;
    A.cx = std::isfinite(x_lo) && std::isfinite(x_hi) ? 0.5 * (x_lo + x_hi) : 0.5 * P.nx;
    A.cy = 0.5;
    double* rho = c->g[c->cur ^ 1];  // the idle population buffer serves as scratch
    hipError_t e = lbm::launch_rho_psi(P, c->g[c->cur], c->psi, rho, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "observables psi");
    e = lbm::launch_obs(P, c->g[c->cur], rho, c->psi, c->gw, A, c->part, c->fin, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "observables");
    double q[32];
    e = hipMemcpyAsync(q, c->fin, lbm::OBS_NQ * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "observables copy");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "observables sync");

    enum { O_MIN = 0, O_MAX, O_U, O_UL, O_MASS, O_BAD, O_N, O_SX, O_SY, O_SXX, O_SYY, O_SXY,
           O_SXR, O_SYR, O_SR };
    lbm_obs o{};
    o.step = c->step;
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
        const double cth = (0.5 - o.yc) / r;
        if (std::isfinite(cth) && std::fabs(cth) <= 1.0) o.theta_deg = std::acos(cth) * 180.0 / M_PI;
    }
    *out = o;
    return o.nonfinite ? LBM_E_NONFINITE : LBM_OK;
}

int lbm_observables(lbm_ctx* c, lbm_obs* out) {
    return lbm_observables_window(c, -INFINITY, INFINITY, out);
}

static int copy_field_out(lbm_ctx* c, const double* dev, int planes, double* host) {
    const KParams& P = c->kp;
    for (int a = 0; a < planes; ++a) {
        hipError_t e = hipMemcpy2DAsync(host + (size_t)a * P.nx * P.ny, P.nx * sizeof(double),
                                        dev + a * P.plane, P.pitch * sizeof(double),
                                        P.nx * sizeof(double), P.ny, hipMemcpyDeviceToHost,
                                        c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "copy out");
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy out sync");
    return LBM_OK;
}

int lbm_read_rho(lbm_ctx* c, double* host, size_t count) {
    if (!c || !host) return LBM_E_INVAL;
    if (count < (size_t)c->p.nx * c->p.ny) return LBM_E_SIZE;
    double* scratch = c->g[c->cur ^ 1];
    hipError_t e = hipMemsetAsync(scratch, 0, (size_t)c->kp.plane * sizeof(double), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "read_rho memset");
    e = lbm::launch_rho_psi(c->kp, c->g[c->cur], c->psi, scratch, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "read_rho");
    return copy_field_out(c, scratch, 1, host);
}

int lbm_read_f(lbm_ctx* c, double* host, size_t count) {
    if (!c || !host) return LBM_E_INVAL;
    if (count < (size_t)9 * c->p.nx * c->p.ny) return LBM_E_SIZE;
    double* scratch = c->g[c->cur ^ 1];
    hipError_t e = hipMemsetAsync(scratch, 0, (size_t)9 * c->kp.plane * sizeof(double), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "read_f memset");
    e = lbm::launch_pull(c->kp, c->g[c->cur], scratch, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "read_f");
    return copy_field_out(c, scratch, 9, host);
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
    return copy_field_out(c, c->g[c->cur], 9, (double*)((char*)host + sizeof h));
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
    for (int a = 0; a < 9; ++a) {
        hipError_t e = hipMemcpy2DAsync(c->g[c->cur] + a * P.plane, P.pitch * sizeof(double),
                                        src + (size_t)a * P.nx * P.ny, P.nx * sizeof(double),
                                        P.nx * sizeof(double), P.ny, hipMemcpyHostToDevice,
                                        c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "load_state");
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "load_state sync");
    c->step = h.step;
    return LBM_OK;
}

int lbm_set_gw(lbm_ctx* c, const double* gw_host) {
    if (!c || !gw_host) return LBM_E_INVAL;
    for (int i = 0; i < 2 * c->p.nx; ++i)
        if (!std::isfinite(gw_host[i])) return fail(c, LBM_E_INVAL, "non-finite G_w");
    hipError_t e = hipMemcpy2DAsync(c->gw, c->kp.pitch * sizeof(double), gw_host,
                                    c->p.nx * sizeof(double), c->p.nx * sizeof(double), 2,
                                    hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_gw");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "set_gw sync");
    return LBM_OK;
}

int lbm_destroy(lbm_ctx* c) {
    if (!c) return LBM_E_INVAL;
    delete c;
    return LBM_OK;
}

}  // extern "C"
