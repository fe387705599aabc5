// tile_emu.cpp -- CPU emulation of the step kernels' workgroups, to check their index maps.
//
// The library's device functions (lbm_device.h) are compiled for the host against the stand-in
// header in tests/emu/hip; a workgroup is emulated by one host thread per device thread with a
// real barrier for __syncthreads. Every launch runs with poisoned memory:
//   * global buffers hold NaN in every slot that is not state (row padding, solid nodes, solid
//     rows except the wet-node force slots), the output buffer is all NaN before the launch;
//   * the LDS of every workgroup is filled with NaN (link words: all bits set) before its tile.
// A read of a slot that was never written therefore turns the result into NaN, and the build
// runs under AddressSanitizer and UndefinedBehaviorSanitizer, which stop at any access outside
// the buffers. Each launch is then checked: every state slot of the output written and finite,
// every other slot untouched, and the two-steps-per-launch kernels (every output tile shape,
// interior and edge tiles) bit for bit equal to two single fused steps. The psi pass and the
// per-node observables are run the same way and must produce finite sums. On periodic and
// bounce-back lattices the adjoint's kernels run too: the segment recomputation (two steps with
// the first written) must equal two fused steps, and one reverse step must write every output
// on the fluid nodes only, bit-equal between the generic tile everywhere and 32 x 4 and 64 x 4
// tiles that take the interior variant where it applies.
//
// Test infrastructure: built and run by tests/test_emu_index_maps.py. Usage:
//   tile_emu            run the built-in case list
//   tile_emu NX NY WALLS GHOST EOS FORCE   run one lattice (WALLS 0..3, EOS 0 CS / 1 Eq. 15)
#include <algorithm>
#include <atomic>
#include <barrier>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

// The device functions under test; a test may point LBM_DEVICE_HEADER at an edited copy.
#ifdef LBM_DEVICE_HEADER
#include LBM_DEVICE_HEADER
#else
#include "../../paper_1410_2569_amd/csrc/lbm_device.h"
#endif

thread_local EmuIdx threadIdx;

namespace {
std::barrier<>* g_bar = nullptr;
std::atomic<int> g_or[3];
thread_local int g_or_gen = 0;
}  // namespace

void __syncthreads() { g_bar->arrive_and_wait(); }

// Three accumulators used in rotation: the one of the previous call is cleared after this
// call's barrier, when every thread has read it and none can reach its next use.
int __syncthreads_or(int v) {
    const int g = g_or_gen;
    g_or_gen = (g + 1) % 3;
    if (v) g_or[g].fetch_or(1);
    g_bar->arrive_and_wait();
    const int r = g_or[g].load();
    if (threadIdx.x == 0) g_or[(g + 2) % 3].store(0);
    return r;
}

namespace {

using lbm::KParams;
const double kNaN = std::numeric_limits<double>::quiet_NaN();
int g_failures = 0;
std::string g_case;

void fail(const std::string& what) {
    ++g_failures;
    std::fprintf(stderr, "FAIL [%s] %s\n", g_case.c_str(), what.c_str());
}

// A pool of host threads, one per device thread of the largest workgroup, reused by every
// emulated launch. run_workgroups() runs tile_fn(k) for k = 0 .. ntiles-1 on an emulated
// workgroup of nthreads threads; before_tile() (one thread, between barriers) re-poisons the
// workgroup's LDS.
class Pool {
  public:
    explicit Pool(int n) {
        for (int t = 0; t < n; ++t) th_.emplace_back([this, t] { worker(t); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& x : th_) x.join();
    }
    void run(int nthreads, int ntiles, const std::function<void(int)>& tile_fn,
             const std::function<void()>& before_tile) {
        std::barrier<> bar(nthreads);
        std::unique_lock<std::mutex> lk(m_);
        job_ = Job{nthreads, ntiles, &tile_fn, &before_tile, &bar};
        for (auto& o : g_or) o.store(0);
        g_bar = &bar;
        active_ = (int)th_.size();
        ++gen_;
        cv_.notify_all();
        done_.wait(lk, [&] { return active_ == 0; });
        g_bar = nullptr;
    }

  private:
    struct Job {
        int nthreads, ntiles;
        const std::function<void(int)>* tile_fn;
        const std::function<void()>* before_tile;
        std::barrier<>* bar;
    };
    void worker(int t) {
        threadIdx.x = (unsigned)t;
        int seen = 0;
        for (;;) {
            std::unique_lock<std::mutex> lk(m_);
            cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
            if (stop_) return;
            seen = gen_;
            const Job j = job_;
            lk.unlock();
            if (t < j.nthreads) {
                g_or_gen = 0;
                for (int k = 0; k < j.ntiles; ++k) {
                    j.bar->arrive_and_wait();
                    if (t == 0) (*j.before_tile)();
                    j.bar->arrive_and_wait();
                    (*j.tile_fn)(k);
                }
            }
            lk.lock();
            if (--active_ == 0) done_.notify_one();
        }
    }
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, done_;
    Job job_{};
    int gen_ = 0, active_ = 0;
    bool stop_ = false;
};

Pool* g_pool = nullptr;

void run_workgroups(int nthreads, int ntiles, const std::function<void(int)>& tile_fn,
                    const std::function<void()>& before_tile) {
    g_pool->run(nthreads, ntiles, tile_fn, before_tile);
}

struct Lattice {
    KParams P{};
    std::vector<unsigned short> links;  // mask: [ny][pitch]
    std::vector<double> gw;             // [2][pitch], or [ny][pitch] per node with a mask
    std::vector<char> state;            // [9][ny][pitch]: slot holds state
    std::vector<char> fluid;            // [ny][pitch]
};

unsigned long long mix(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
double unit(unsigned long long k) { return (mix(k) >> 11) * 0x1.0p-53; }

Lattice make_lattice(int nx, int ny, int walls, int ghost, int eos, int wall_force) {
    Lattice L;
    KParams& k = L.P;
    k.nx = nx;
    k.ny = ny;
    k.pitch = (nx + 31) / 32 * 32;
    k.plane = (long long)ny * k.pitch;
    k.walls = walls;
    k.ghost = walls == 3 ? 0 : ghost;
    k.wet = walls == 2;
    k.mask = walls == 3;
    k.eos = eos;
    k.wall_force = wall_force;
    k.y_lo = (walls == 1 || walls == 2) ? 1 : 0;
    k.y_hi = (walls == 1 || walls == 2) ? ny - 2 : ny - 1;
    double rho_l, rho_v, sigma;
    if (eos == 0) {  // Carnahan-Starling at density ratio 500
        k.RT = 0.0244618784;
        k.a = 0.5;
        k.b4 = 1.0;
        rho_v = 8.901265e-4;
        rho_l = 0.4450633;
        sigma = 0.11244;
    } else {  // Eq. (15) at (1, 500)
        k.th_v = 0.64 / 3.0;
        k.th_m = -0.04 / 3.0;
        k.th_l = 1.0 / 3.0;
        k.rho1 = 1.3585916;
        k.rho2 = 481.04216;
        k.p1 = k.rho1 * k.th_v;
        k.p2 = k.p1 + (k.rho2 - k.rho1) * k.th_m;
        rho_v = 1.0;
        rho_l = 500.0;
        sigma = 0.084;
    }
    k.two_over_G = -2.0;
    k.negG = 1.0;
    k.rho_mid = 0.5 * (rho_l + rho_v);
    k.c_sig_e = k.c_sig_z = 12.0 * sigma / (1.25 - 0.5);
    k.s_e = k.s_z = 0.8;
    k.s_j = 1.0;
    k.s_q = 1.1;
    k.h_e = k.h_z = 0.6;
    k.h_j = 0.5;
    k.h_q = 0.45;
    const double nu_l = 0.1 / 3.0, nu_v = 1.5 / 3.0;  // tau 0.6 and 2.0: interpolated shear rate
    k.visc_const = 0;
    k.nu_v = nu_v;
    k.dnu = nu_l - nu_v;
    k.rho_v = rho_v;
    k.inv_drho = 1.0 / (rho_l - rho_v);
    k.s_nu_c = 1.0 / (3.0 * nu_v + 0.5);

    const int pitch = k.pitch;
    L.fluid.assign((size_t)ny * pitch, 0);
    if (walls == 3) {
        // pillars of height min(3, ny/4), 2 wide with gaps of 1, on a base row and under a top row
        std::vector<char> solid((size_t)ny * nx, 0);
        const int h = std::max(1, std::min(3, ny / 4));
        for (int x = 0; x < nx; ++x) {
            solid[x] = 1;
            solid[(size_t)(ny - 1) * nx + x] = 1;
            if (x % 3 != 2)
                for (int y = 1; y <= h && y < ny - 2; ++y) solid[(size_t)y * nx + x] = 1;
        }
        static const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        static const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        L.links.assign((size_t)ny * pitch, 1);
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                unsigned short w = 0;
                for (int a = 0; a < 9; ++a) {
                    const int xs = ((x - ex[a]) % nx + nx) % nx, ys = ((y - ey[a]) % ny + ny) % ny;
                    if (solid[(size_t)ys * nx + xs]) w |= (unsigned short)(1u << a);
                }
                L.links[(size_t)y * pitch + x] = w;
                L.fluid[(size_t)y * pitch + x] = !solid[(size_t)y * nx + x];
            }
        L.gw.assign((size_t)ny * pitch, kNaN);
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                if (solid[(size_t)y * nx + x]) L.gw[(size_t)y * pitch + x] = 0.05 * (2 * unit(7 * y + x) - 1);
        k.links = L.links.data();
        k.gwn = L.gw.data();
    } else {
        for (int y = k.y_lo; y <= k.y_hi; ++y)
            for (int x = 0; x < nx; ++x) L.fluid[(size_t)y * pitch + x] = 1;
        L.gw.assign((size_t)2 * pitch, kNaN);
        for (int r = 0; r < 2; ++r)
            for (int x = 0; x < nx; ++x) L.gw[(size_t)r * pitch + x] = 0.05 * (2 * unit(1000 + 2 * x + r) - 1);
    }
    L.state.assign((size_t)9 * k.plane, 0);
    for (int a = 0; a < 9; ++a)
        for (size_t i = 0; i < (size_t)k.plane; ++i) L.state[a * k.plane + i] = L.fluid[i];
    if (walls == 2)  // wet-node force of the boundary nodes: planes 0 and 1 of the solid rows
        for (int a = 0; a < 2; ++a)
            for (int x = 0; x < nx; ++x) {
                L.state[a * k.plane + x] = 1;
                L.state[a * k.plane + (size_t)(ny - 1) * pitch + x] = 1;
            }
    return L;
}

// A smooth density within one phase (so that two steps stay inside the EOS domain whatever the
// geometry) with a little noise on every population, so that a population read from the wrong
// slot changes the result; wet-node force slots get small values; NaN outside the state.
std::vector<double> make_state(const Lattice& L) {
    const KParams& k = L.P;
    // without ghost rows a solid row pulls the liquid next to it by psi_L^2 / 3: vapour then
    const bool vap = k.walls && !k.ghost;
    const double base = k.eos == 0 ? (vap ? 0.02 : 0.40) : (vap ? 1.0 : 400.0);
    const double t9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    std::vector<double> g((size_t)9 * k.plane, kNaN);
    for (int y = 0; y < k.ny; ++y)
        for (int x = 0; x < k.nx; ++x) {
            const size_t i = (size_t)y * k.pitch + x;
            const double rho = base * (1.0 + 0.08 * std::sin(6.283185307179586 * x / k.nx) *
                                                 std::cos(6.283185307179586 * y / k.ny));
            for (int a = 0; a < 9; ++a) {
                if (!L.state[a * k.plane + i]) continue;
                const double n = 2.0 * unit(((unsigned long long)a << 40) + i) - 1.0;
                g[a * k.plane + i] = L.fluid[i] ? t9[a] * rho * (1.0 + 0.02 * n) : 1e-4 * n;
            }
        }
    return g;
}

template <int GEO, int EOS, int TX = 64, int TY = 4>
void step_fused(const Lattice& L, const double* gin, double* gout) {
    const KParams& P = L.P;
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.y_hi - P.y_lo + TY) / TY;
    std::vector<double> sp((TY + 2) * (TX + 2));
    run_workgroups(
        TX * TY, ntx * nty,
        [&](int t) {
            lbm::step_tile<TX, TY, true, GEO, EOS>(P, gin, gout, nullptr, L.gw.data(),
                                                   (t % ntx) * TX, P.y_lo + (t / ntx) * TY,
                                                   sp.data());
        },
        [&] { std::fill(sp.begin(), sp.end(), kNaN); });
}

template <int TX, int TY, int GEO, int EOS, int NTH = lbm::step2_threads(TX, TY, GEO)>
void step_two(const Lattice& L, const double* gin, double* gout) {
    const KParams& P = L.P;
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.y_hi - P.y_lo + TY) / TY;
    auto* lds = new lbm::Step2Lds<TX, TY, GEO>;
    run_workgroups(
        NTH, ntx * nty,
        [&](int t) {
            lbm::step2_tile_any<TX, TY, GEO, EOS, false, false, NTH>(
                P, gin, gout, L.gw.data(), (t % ntx) * TX, P.y_lo + (t / ntx) * TY, *lds);
        },
        [&] { std::memset((void*)lds, 0xFF, sizeof *lds); });
    delete lds;
}

// Output checks: state slots written and finite, every other slot still NaN.
void check_output(const Lattice& L, const std::vector<double>& g, const char* what) {
    size_t unwritten = 0, stray = 0;
    for (size_t i = 0; i < g.size(); ++i) {
        if (L.state[i]) unwritten += !std::isfinite(g[i]);
        else stray += !std::isnan(g[i]);
    }
    if (unwritten) fail(std::string(what) + ": " + std::to_string(unwritten) + " state slots not finite");
    if (stray) fail(std::string(what) + ": " + std::to_string(stray) + " non-state slots written");
}

void check_equal(const Lattice& L, const std::vector<double>& a, const std::vector<double>& b,
                 const char* what) {
    size_t diff = 0;
    for (size_t i = 0; i < a.size(); ++i)
        if (L.state[i] && std::memcmp(&a[i], &b[i], sizeof(double)) != 0) ++diff;
    if (diff) fail(std::string(what) + ": " + std::to_string(diff) + " slots differ from two fused steps");
}

// Two steps with the intermediate state written (the segment recomputation of the adjoint).
template <int TX, int TY, int EOS, int NTH = lbm::step2_threads(TX, TY, lbm::GEO_ROWS)>
void step_two_mid(const Lattice& L, const double* gin, double* gout, double* gmid) {
    const KParams& P = L.P;
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.y_hi - P.y_lo + TY) / TY;
    auto* lds = new lbm::Step2Lds<TX, TY, lbm::GEO_ROWS>;
    run_workgroups(
        NTH, ntx * nty,
        [&](int t) {
            lbm::step2_tile_any<TX, TY, lbm::GEO_ROWS, EOS, true, false, NTH>(
                P, gin, gout, L.gw.data(), (t % ntx) * TX, P.y_lo + (t / ntx) * TY, *lds, gmid);
        },
        [&] { std::memset((void*)lds, 0xFF, sizeof *lds); });
    delete lds;
}

// One reverse step (adj_tile) on TX x TY tiles.
struct AdjBufs {
    std::vector<double> a_in, q_in, p0_in, dpsi_in, rv_in, a_out, q_out, p0_out, dpsi_out, rv_out,
        gg;
};

// MODE 0: adj_tile (interior variant where it applies), 1: every tile the generic variant.
template <int TX, int TY, int NTH = TX * TY, int EOS = lbm::EOS_ANY, int MODE = 0>
void adj_step(const Lattice& L, const double* gprev, AdjBufs& B) {
    const KParams& P = L.P;
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.y_hi - P.y_lo + TY) / TY;
    auto* lds = new lbm::AdjLds<TX, TY>;
    const lbm::AdjPtrs A{gprev,           B.a_in.data(),  B.q_in.data(),  B.p0_in.data(),
                         B.dpsi_in.data(), B.rv_in.data(), L.gw.data(),    B.a_out.data(),
                         B.q_out.data(),  B.p0_out.data(), B.dpsi_out.data(), B.rv_out.data(),
                         B.gg.data()};
    run_workgroups(
        NTH, ntx * nty,
        [&](int t) {
            const int x0 = (t % ntx) * TX, y0 = P.y_lo + (t / ntx) * TY;
            if constexpr (MODE == 0) lbm::adj_tile<TX, TY, NTH, EOS>(P, A, x0, y0, *lds);
            else lbm::adj_tile_impl<TX, TY, NTH, EOS, false>(P, A, x0, y0, *lds);
        },
        [&] { std::fill((double*)lds, (double*)lds + sizeof *lds / sizeof(double), kNaN); });
    delete lds;
}

// Later-step adjoint inputs: small seeded values on the fluid nodes (psi' > 0), NaN elsewhere;
// outputs NaN; the G_w gradient zero on its two rows.
AdjBufs make_adj(const Lattice& L) {
    const KParams& P = L.P;
    const size_t pl = (size_t)P.plane;
    AdjBufs B;
    auto fill = [&](std::vector<double>& v, int planes, unsigned long long salt, double lo,
                    double hi) {
        v.assign(planes * pl, kNaN);
        for (int k = 0; k < planes; ++k)
            for (size_t i = 0; i < pl; ++i)
                if (L.fluid[i]) v[k * pl + i] = lo + (hi - lo) * unit((salt << 48) + k * pl + i);
    };
    fill(B.a_in, 9, 1, -1.0, 1.0);
    fill(B.q_in, 2, 2, -0.5, 0.5);
    fill(B.p0_in, 1, 3, -0.5, 0.5);
    fill(B.dpsi_in, 1, 4, 0.5, 1.5);
    B.rv_in.assign((size_t)4 * P.pitch, kNaN);
    for (int r = 0; r < 4; ++r)
        for (int x = 0; x < P.nx; ++x) B.rv_in[(size_t)r * P.pitch + x] = unit(5000 + 4 * x + r) - 0.5;
    B.a_out.assign(9 * pl, kNaN);
    B.q_out.assign(2 * pl, kNaN);
    B.p0_out.assign(pl, kNaN);
    B.dpsi_out.assign(pl, kNaN);
    B.rv_out.assign((size_t)4 * P.pitch, kNaN);
    B.gg.assign((size_t)2 * P.pitch, kNaN);
    for (int r = 0; r < 2; ++r)
        for (int x = 0; x < P.nx; ++x) B.gg[(size_t)r * P.pitch + x] = 0.0;
    return B;
}

// Adjoint outputs written and finite exactly on the fluid nodes (wall vectors and G_w gradient:
// on their rows when there are walls), and bit-equal between two tile shapes.
void check_adj(const Lattice& L, const AdjBufs& X, const AdjBufs& Y, const char* what) {
    const KParams& P = L.P;
    const size_t pl = (size_t)P.plane;
    size_t bad = 0, stray = 0, diff = 0;
    auto node = [&](const std::vector<double>& v, const std::vector<double>& w, int planes) {
        for (int k = 0; k < planes; ++k)
            for (size_t i = 0; i < pl; ++i) {
                const double a = v[k * pl + i];
                if (L.fluid[i]) bad += !std::isfinite(a);
                else stray += !std::isnan(a);
                diff += std::memcmp(&a, &w[k * pl + i], sizeof(double)) != 0;
            }
    };
    node(X.a_out, Y.a_out, 9);
    node(X.q_out, Y.q_out, 2);
    node(X.p0_out, Y.p0_out, 1);
    node(X.dpsi_out, Y.dpsi_out, 1);
    for (int r = 0; r < 4; ++r)
        for (int x = 0; x < P.pitch; ++x) {
            const size_t i = (size_t)r * P.pitch + x;
            const double a = X.rv_out[i];
            if (P.walls && x < P.nx) bad += !std::isfinite(a);
            else stray += !std::isnan(a);
            diff += std::memcmp(&a, &Y.rv_out[i], sizeof(double)) != 0;
        }
    for (size_t i = 0; i < X.gg.size(); ++i) {
        bad += (i % P.pitch) < (size_t)P.nx && !std::isfinite(X.gg[i]);
        diff += std::memcmp(&X.gg[i], &Y.gg[i], sizeof(double)) != 0;
    }
    if (bad) fail(std::string(what) + ": " + std::to_string(bad) + " outputs not finite");
    if (stray) fail(std::string(what) + ": " + std::to_string(stray) + " slots written off the fluid");
    if (diff) fail(std::string(what) + ": " + std::to_string(diff) + " outputs differ between tile shapes");
}

template <int EOS>
void run_adjoint(const Lattice& L, const std::vector<double>& g0, const std::vector<double>& g1,
                 const std::vector<double>& g2) {
    // segment recomputation: two steps with the first written, against two fused steps
    for (int shape = 0; shape < 3; ++shape) {
        std::vector<double> mid(g0.size(), kNaN), out(g0.size(), kNaN);
        const char* name = shape == 2 ? "two-step 64x4 wide + mid"
                                      : (shape ? "two-step 64x8 + mid" : "two-step 64x4 + mid");
        if (shape == 2)
            step_two_mid<64, 4, EOS, lbm::step2_wide_threads(64, 4)>(L, g0.data(), out.data(),
                                                                    mid.data());
        else if (shape) step_two_mid<64, 8, EOS>(L, g0.data(), out.data(), mid.data());
        else step_two_mid<64, 4, EOS>(L, g0.data(), out.data(), mid.data());
        check_output(L, mid, name);
        check_equal(L, mid, g1, name);
        check_output(L, out, name);
        check_equal(L, out, g2, name);
    }
    // one reverse step: the generic tile everywhere (32 x 4), against 64 x 4 tiles and 32 x 4
    // tiles with two threads per node, both with the interior variant where it applies and the
    // equation of state fixed at compile time
    AdjBufs X = make_adj(L), Y = make_adj(L), Z = make_adj(L);
    adj_step<32, 4, 128, lbm::EOS_ANY, 1>(L, g0.data(), X);
    adj_step<64, 4, 256, EOS>(L, g0.data(), Y);
    adj_step<32, 4, 256, EOS>(L, g0.data(), Z);
    check_adj(L, X, Y, "reverse step: generic 32x4 vs 64x4 (interior variant)");
    check_adj(L, X, Z, "reverse step: generic 32x4 vs 32x4, 256 threads (interior variant)");
}

template <int GEO, int EOS>
void observables(const Lattice& L, const std::vector<double>& g) {
    const KParams& P = L.P;
    std::vector<double> psi((size_t)P.plane, kNaN), rho((size_t)P.plane, kNaN);
    if (P.walls && !P.mask && !P.ghost)  // never written: the workspace is zeroed at creation
        for (int x = 0; x < P.nx; ++x) psi[x] = psi[(size_t)(P.ny - 1) * P.pitch + x] = 0.0;
    for (int y = P.y_lo; y <= P.y_hi; ++y)
        for (int x = 0; x < P.nx; ++x) lbm::psi_node(P, g.data(), psi.data(), rho.data(), x, y);
    lbm::ObsArgs A{P.rho_mid, 3.5, -INFINITY, INFINITY, 0.5 * P.nx, 0.5};
    double tot[lbm::O_NQ];
    for (int q = 0; q < lbm::O_NQ; ++q) tot[q] = lbm::op_identity(q);
    for (int y = P.y_lo; y <= P.y_hi; ++y)
        for (int x = 0; x < P.nx; ++x) {
            double v[lbm::O_NQ];
            for (int q = 0; q < lbm::O_NQ; ++q) v[q] = lbm::op_identity(q);
            lbm::obs_node(P, g.data(), rho.data(), psi.data(), L.gw.data(), A, x, y, v);
            for (int q = 0; q < lbm::O_NQ; ++q) tot[q] = lbm::op_combine(q, tot[q], v[q]);
        }
    for (int q = 0; q < lbm::O_NQ; ++q)
        if (!std::isfinite(tot[q]) && !(q == lbm::O_UL && tot[q] == -INFINITY))
            fail("observables: quantity " + std::to_string(q) + " not finite");
    if (tot[lbm::O_BAD] != 0.0) fail("observables: non-finite nodes");
}

template <int GEO, int EOS>
void run_case(const Lattice& L) {
    const std::vector<double> g0 = make_state(L);
    // reference: two single fused steps
    std::vector<double> g1(g0.size(), kNaN), ref(g0.size(), kNaN);
    step_fused<GEO, EOS>(L, g0.data(), g1.data());
    check_output(L, g1, "fused step 1");
    step_fused<GEO, EOS>(L, g1.data(), ref.data());
    check_output(L, ref, "fused step 2");
    {  // the fused step on 32 x 4 tiles (the odd step of an ensemble on that work-list)
        std::vector<double> g1n(g0.size(), kNaN);
        step_fused<GEO, EOS, 32, 4>(L, g0.data(), g1n.data());
        check_output(L, g1n, "fused step 32x4");
        check_equal(L, g1n, g1, "fused step 32x4");
    }
    auto two = [&](auto fn, const char* name) {
        std::vector<double> out(g0.size(), kNaN);
        fn(L, g0.data(), out.data());
        check_output(L, out, name);
        check_equal(L, out, ref, name);
    };
    two(step_two<64, 8, GEO, EOS>, "two-step 64x8");
    two(step_two<64, 8, GEO, EOS, 512>, "two-step 64x8, 512 threads");
    two(step_two<64, 4, GEO, EOS>, "two-step 64x4");
    two(step_two<128, 4, GEO, EOS>, "two-step 128x4");
    two(step_two<64, 16, GEO, EOS>, "two-step 64x16");
    two(step_two<32, 8, GEO, EOS>, "two-step 32x8");
    two(step_two<32, 4, GEO, EOS>, "two-step 32x4");
    two(step_two<64, 4, GEO, EOS, lbm::step2_wide_threads(64, 4)>, "two-step 64x4, wide");
    two(step_two<32, 4, GEO, EOS, lbm::step2_wide_threads(32, 4)>, "two-step 32x4, wide");
    observables<GEO, EOS>(L, ref);
    if constexpr (GEO == lbm::GEO_ROWS) run_adjoint<EOS>(L, g0, g1, ref);
}

void run_lattice(int nx, int ny, int walls, int ghost, int eos, int force) {
    char buf[128];
    std::snprintf(buf, sizeof buf, "%dx%d walls=%d ghost=%d eos=%d force=%d", nx, ny, walls, ghost,
                  eos, force);
    g_case = buf;
    Lattice L = make_lattice(nx, ny, walls, ghost, eos, force);
    if (L.P.mask) {  // the kernel parameters point into the lattice's own arrays
        L.P.links = L.links.data();
        L.P.gwn = L.gw.data();
    }
    const int geo = walls == 3 ? lbm::GEO_MASK : (walls == 2 ? lbm::GEO_WET : lbm::GEO_ROWS);
    const int before = g_failures;
    if (geo == lbm::GEO_MASK) {
        eos ? run_case<lbm::GEO_MASK, lbm::EOS_PW>(L) : run_case<lbm::GEO_MASK, lbm::EOS_CS>(L);
    } else if (geo == lbm::GEO_WET) {
        eos ? run_case<lbm::GEO_WET, lbm::EOS_PW>(L) : run_case<lbm::GEO_WET, lbm::EOS_CS>(L);
    } else {
        eos ? run_case<lbm::GEO_ROWS, lbm::EOS_PW>(L) : run_case<lbm::GEO_ROWS, lbm::EOS_CS>(L);
    }
    std::printf("%s %s\n", g_failures == before ? "ok  " : "FAIL", buf);
    std::fflush(stdout);
}

}  // namespace

int main(int argc, char** argv) {
    Pool pool(1024);  // the largest workgroup: two-step 64 x 16 tiles
    g_pool = &pool;
    if (argc == 7) {
        run_lattice(std::atoi(argv[1]), std::atoi(argv[2]), std::atoi(argv[3]), std::atoi(argv[4]),
                    std::atoi(argv[5]), std::atoi(argv[6]));
        return g_failures ? 1 : 0;
    }
    // lattices from 3 x 4 to 125 x 17 (ragged tiles, several halo wraps, rows of width 1 in x
    // modulo the tile), and two with interior tiles
    const int sizes[][2] = {{3, 4},   {4, 5},    {7, 6},    {17, 9},   {33, 10}, {63, 12},
                            {64, 12}, {65, 13},  {125, 17}, {130, 30}, {200, 40}};
    int k = 0;
    for (const auto& s : sizes) {
        for (int walls = 0; walls <= 3; ++walls) {
            if (walls == 3 && s[1] < 6) continue;  // pillars need a few rows
            const int force = k % 3;
            run_lattice(s[0], s[1], walls, 1, k % 4 == 3 ? 1 : 0, force);
            if (walls == 1) run_lattice(s[0], s[1], walls, 0, 0, (force + 1) % 3);
            ++k;
        }
    }
    std::printf("%s: %d failure(s)\n", g_failures ? "FAILED" : "passed", g_failures);
    return g_failures ? 1 : 0;
}
