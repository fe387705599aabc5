/*
 * lbm.h -- C ABI of liblbm: one GPU time step of the D2Q9 multi-relaxation-time pseudopotential
 * (Shan-Chen) lattice Boltzmann model of wetting at large density ratio, with the three
 * fluid-solid adhesion forces compared by Q. Li, K. H. Luo, Q. J. Kang and Q. Chen, "Contact
 * angles in the pseudopotential lattice Boltzmann modeling of wetting" (2014).
 *
 * Conventions for every entry point
 * ---------------------------------
 * - All functions are extern "C", return int: LBM_OK (0) or a negative LBM_E_* code. They never
 *   abort or exit. lbm_strerror() names a code; lbm_last_error() gives the message of the last
 *   failure on a context, or with NULL that of the last failed creation on the calling thread.
 * - Arithmetic is IEEE binary64 throughout.
 * - Lattice: nx columns (x, periodic) by ny rows (y). With walls = 1 or 2, rows y = 0 and
 *   y = ny-1 are solid nodes (flat walls) and the fluid occupies rows 1 .. ny-2. walls = 1:
 *   halfway bounce-back, wall planes at y = 0.5 and y = ny - 1.5. walls = 2: the non-slip
 *   wet-node scheme of Sec. III.A, wall planes on the boundary nodes y = 1 and y = ny - 2. With
 *   walls = 0, y is periodic too.
 * - Host arrays are row-major with x fastest: a field is [ny][nx]; populations are [9][ny][nx]
 *   in the velocity order 0 rest; 1..4 = E, N, W, S; 5..8 = NE, NW, SW, SE.
 * - Wall wettability G_w is given per solid node: gw[2][nx], row 0 for the bottom wall (y = 0),
 *   row 1 for the top wall (y = ny-1).
 * - Device memory: the library never allocates device memory. The caller passes one device
 *   workspace of at least lbm_workspace_size() bytes; it must stay allocated until
 *   lbm_destroy(). The library keeps f, psi, G_w and reduction partials inside it.
 * - Streams: a context is bound to the hipStream_t given at creation (NULL = default stream).
 *   Stepping calls are asynchronous on that stream; calls that return host data synchronise
 *   it. A context is not thread-safe.
 * - Parameters are validated before any HIP call, so invalid input is reported without a GPU.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 1

enum {
    LBM_OK = 0,
    LBM_E_INVAL = -1,     /* invalid argument or parameter */
    LBM_E_SIZE = -2,      /* workspace or host buffer too small */
    LBM_E_HIP = -3,       /* a HIP runtime call failed */
    LBM_E_NONFINITE = -4, /* NaN/Inf or an undefined pseudopotential found in the state */
    LBM_E_ABI = -5,       /* abi_version mismatch */
    LBM_E_STATE = -6      /* state blob does not match this context */
};

/* Adhesion force (pre-sum factor of the fluid-solid interaction):
 * density-based Eq. (10), pseudopotential-based Eq. (11), modified pseudopotential-based Eq. (14). */
enum lbm_wall { LBM_WALL_RHO = 0, LBM_WALL_PSI = 1, LBM_WALL_MODPSI = 2 };

/* Equation of state feeding psi = sqrt(2 (p_EOS - rho c_s^2) / (G c^2)) (Sec. II.B):
 * Carnahan-Starling p = rho R T (1 + eta + eta^2 - eta^3)/(1 - eta)^3 - a rho^2, eta = b rho / 4,
 * or the piecewise-linear Eq. (15) of Sec. III. */
enum lbm_eos { LBM_EOS_CS = 0, LBM_EOS_PIECEWISE = 1 };

/* Geometry in y (lbm_params.walls).
 * LBM_WALLS_BOUNCE_BACK: a population that would stream in from a solid node is the one the node
 *   itself sent towards the wall (halfway bounce-back).
 * LBM_WALLS_WET_NODE: the non-slip boundary of Sec. III.A. The boundary nodes (rows 1 and ny-2)
 *   reconstruct the populations arriving from the solid from the streamed ones and their force
 *   F of the previous step so that sum_a e_a f_a + F/2 = 0 (bottom wall: f2 = f4,
 *   f5 = f7 - (f1 - f3)/2 - (Fx + Fy)/4, f6 = f8 + (f1 - f3)/2 + (Fx - Fy)/4; the top wall is the
 *   same rule rotated by 180 degrees). That force is part of the state (saved with it).
 * LBM_WALLS_MASK: periodic in x and y with an arbitrary solid mask (rough surfaces, Sec. III.B),
 *   given to lbm_create_masked: halfway bounce-back on every link from a solid node, psi = 0 on
 *   solid nodes (Eq. 7 is not applied across the solid, so ghost_psi must be 0) and G_w per
 *   solid node. */
enum lbm_geometry { LBM_PERIODIC = 0, LBM_WALLS_BOUNCE_BACK = 1, LBM_WALLS_WET_NODE = 2,
                    LBM_WALLS_MASK = 3 };

typedef struct {
    int32_t abi_version; /* must be LBM_ABI_VERSION */
    int32_t nx, ny;      /* nx >= 3; ny >= 4 with walls, >= 3 without */
    int32_t walls;       /* enum lbm_geometry: 0 periodic in y; 1, 2 solid rows 0 and ny-1 */
    int32_t ghost_psi;   /* 1: Eq. (7) also acts across the wall: a solid row carries the psi of
                            the adjacent fluid row, so G_w = 0 is neutral wetting (Sec. III.A);
                            0: psi = 0 on solid nodes */
    int32_t eos;         /* enum lbm_eos */
    int32_t wall_force;  /* enum lbm_wall */
    int32_t reserved;    /* must be 0 */
    double a, b, R, T;   /* Carnahan-Starling constants */
    double rho1, rho2, th_v, th_m, th_l; /* Eq. (15): spinodal densities and slopes */
    double G;            /* interaction strength of Eq. (7); must be < 0 */
    double sigma;        /* mechanical-stability parameter of the forcing term Eq. (9) */
    double s_rho, s_e, s_zeta, s_j, s_q; /* relaxation rates of Eq. (2), each in (0, 2) */
    double tau_l, tau_v; /* tau_nu in liquid and vapour, each > 1/2; kinematic viscosity
                            nu = (tau_nu - 1/2)/3 is interpolated linearly in the phase fraction
                            (rho - rho_v)/(rho_l - rho_v), clamped to [0, 1] */
    double rho_l, rho_v; /* coexistence densities (rho_l > rho_v > 0): viscosity interpolation,
                            contact-angle contour rho_mid = (rho_l + rho_v)/2 */
} lbm_params;

typedef struct {
    int64_t step;        /* time step n of the observed state f^n */
    double rho_min, rho_max; /* over fluid nodes (Table I of the paper) */
    double umax;         /* max |v| over fluid nodes, v of Eq. (6) (spurious currents, Fig. 9) */
    double umax_liquid;  /* max |v| over nodes with rho >= rho_mid */
    double mass;         /* sum of rho over fluid nodes */
    double theta_deg;    /* static contact angle on the bottom wall, NaN if undefined */
    double xc, yc, r;    /* fitted circle */
    int32_t n_fit;       /* interface points used by the fit */
    int32_t nonfinite;   /* number of fluid nodes with a non-finite rho, psi or v */
} lbm_obs;

typedef struct lbm_ctx lbm_ctx;

/* ---- Thermodynamics (host only, no GPU) --------------------------------------------------- */

/* Maxwell construction (equal-area rule in 1/rho together with p(rho_v) = p(rho_l) = p0) for the
 * Carnahan-Starling EOS at temperature T. LBM_E_INVAL if T is not below the critical point. */
int lbm_maxwell_cs(double a, double b, double R, double T, double *rho_v, double *rho_l,
                   double *p0);
/* Temperature at which the Carnahan-Starling Maxwell densities have ratio rho_l/rho_v = ratio. */
int lbm_cs_temperature(double a, double b, double R, double ratio, double *T);
/* Spinodal densities rho1 < rho2 of the piecewise-linear EOS, Eq. (15), whose Maxwell
 * coexistence densities are (rho_v, rho_l): mechanical and chemical equilibrium as in Sec. III
 * (for (1, 500) and slopes (0.64, -0.04, 1) c_s^2 the paper gives 1.36 and 481.04).
 * LBM_E_INVAL if no such pair exists (needs th_m < th_l and rho_v < rho1 < rho2 < rho_l). */
int lbm_piecewise_spinodals(double rho_v, double rho_l, double th_v, double th_m, double th_l,
                            double *rho1, double *rho2);

/* Equation of state p_EOS(rho) of the parameter block (host only): the bulk pressure of Eq. (8)
 * for the pseudopotential of Sec. II.B. LBM_E_INVAL for invalid parameters or rho outside the
 * EOS domain. */
int lbm_pressure(const lbm_params *p, double rho, double *out);

/* ---- Single instance ---------------------------------------------------------------------- */

/* Bytes of device workspace a context with these parameters needs. */
int lbm_workspace_size(const lbm_params *p, size_t *bytes);

/* Create a context in the caller's workspace d_ws (device pointer, >= lbm_workspace_size()).
 * gw_host: [2][nx] host array of G_w per solid node (may be NULL with walls = 0; copied).
 * rho0_host: [ny][nx] host array of the initial density (solid rows ignored; copied); every
 * fluid value positive and inside the pseudopotential's domain (2 (p_EOS - rho/3) / G >= 0),
 * else LBM_E_INVAL. The initial populations are the rest equilibrium f_a = t_a rho0 with
 * t = 4/9, 1/9, 1/36.
 * stream: hipStream_t (NULL = default). On success *out owns host memory only.
 * walls = LBM_WALLS_MASK is rejected here (LBM_E_INVAL): use lbm_create_masked. */
int lbm_create(const lbm_params *p, const double *gw_host, const double *rho0_host, void *d_ws,
               size_t ws_bytes, void *stream, lbm_ctx **out);

/* Initial state generated on the device: liquid droplets in their vapour (Sec. III: a droplet
 * placed on the wall relaxes to its contact angle; the tanh profile below replaces the sharp
 * step of Eq. 16, which at density ratio 500 starts with a shock). On every fluid node
 *     rho0 = max_k [ (rho_l + rho_v)/2 - (rho_l - rho_v)/2 tanh(2 (d_k - radius[k]) / width) ]
 * with d_k the distance of (x, y) from (x0[k], y0[k]) in lattice units, then, when jitter > 0,
 *     rho0 <- rho0 (1 + jitter (2u - 1)),
 * u = (splitmix64(splitmix64(seed) + y nx + x) >> 11) 2^-53 with S. Vigna's SplitMix64 (all
 * arithmetic modulo 2^64). */
#define LBM_MAX_DROPLETS 64
typedef struct {
    int32_t count;    /* 1 .. LBM_MAX_DROPLETS */
    int32_t reserved; /* must be 0 */
    double x0[LBM_MAX_DROPLETS], y0[LBM_MAX_DROPLETS], radius[LBM_MAX_DROPLETS]; /* radius > 0 */
    double width;     /* > 0 */
    double jitter;    /* 0 <= jitter < 1 (0: none) */
    uint64_t seed;
} lbm_droplets;

/* lbm_create with the initial density of `drops` (copied) computed on the device instead of a
 * host array; walls 0, 1 or 2 (LBM_E_INVAL for a solid mask, an invalid description, or a jitter
 * that would take a density out of the pseudopotential's domain). */
int lbm_create_droplets(const lbm_params *p, const double *gw_host, const lbm_droplets *drops,
                        void *d_ws, size_t ws_bytes, void *stream, lbm_ctx **out);

/* Create a context on an arbitrary solid geometry (p->walls = LBM_WALLS_MASK, ghost_psi = 0;
 * rough surfaces of Sec. III.B). solid_host: [ny][nx] bytes, nonzero = solid node; gw_host:
 * [ny][nx] G_w of every solid node (values on fluid nodes are ignored); rho0_host: [ny][nx]
 * initial density (solid nodes ignored, fluid nodes > 0). All copied. x and y are periodic: a
 * closed channel lists its wall rows in the mask. Such a context runs every schedule but the
 * overlapped fused tiles (lbm_set_schedule); the adjoint entry points reject it.
 * LBM_E_INVAL for any other walls value, a null array or a mask without fluid nodes. */
int lbm_create_masked(const lbm_params *p, const uint8_t *solid_host, const double *gw_host,
                      const double *rho0_host, void *d_ws, size_t ws_bytes, void *stream,
                      lbm_ctx **out);

/* Advance n >= 0 time steps (Eqs. 1-9 with the adhesion force and the context's wall scheme).
 * Asynchronous on the context stream. */
int lbm_step(lbm_ctx *c, int64_t n);

/* Observables of the current state f^n (Sec. III.B, III.C and the contact angle of Figs. 1-4):
 * density extremes, spurious-current maxima, mass, and the contact angle from a Kasa circle fit
 * of the rho_mid contour (crossings on lattice edges with y >= 3.5, the bottom wall plane plus
 * about one interface width). Synchronises the stream. Returns LBM_E_NONFINITE (after filling
 * *out) if any fluid node is not finite. */
int lbm_observables(lbm_ctx *c, lbm_obs *out);

/* Same, with the fit restricted to interface points with x_lo <= x < x_hi (one droplet of
 * several). */
int lbm_observables_window(lbm_ctx *c, double x_lo, double x_hi, lbm_obs *out);

/* Same, with the contact plane at height y_wall (points with y >= y_wall + 3 are fitted and
 * theta = acos((y_wall - yc)/r)): the apparent angle on pillars whose tops end at y_wall. The
 * default plane is y = 0.5 (bounce-back and masked geometries) or 1 (wet-node walls). */
int lbm_observables_plane(lbm_ctx *c, double x_lo, double x_hi, double y_wall, lbm_obs *out);

/* Allocation-free observables, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the record of
 * lbm_observables for a population field the caller already holds on the device, with no context
 * and no workspace.
 *   p      parameters (walls 0, 1 or 2; a solid mask gets LBM_E_INVAL);
 *   d_f    device array [9][ny][nx] of the PRE-collision populations f^n (the layout lbm_read_f
 *          returns), caller-owned, read only, 8-byte aligned;
 *   d_gw   device array [2][nx] of G_w (bottom wall, top wall), caller-owned; may be NULL with
 *          walls = 0;
 *   stream hipStream_t of the current device (NULL = default stream); the call synchronises it;
 *   out    host record, out->step = 0.
 * The density and pseudopotential planes and the partial sums live in a fixed 24 MiB device
 * array of the library (one per GPU, held until the process ends); nothing is allocated. A
 * lattice that needs more (about 1.5 million nodes; 1024 x 1024 fits) gets LBM_E_SIZE, with the
 * reason in lbm_last_error(NULL). Calls that overlap on one GPU (several host threads or streams)
 * share that array and race. Returns LBM_E_NONFINITE (after filling *out) if a fluid node is not
 * finite. */
int lbm_observables_of_state(const lbm_params *p, const double *d_f, const double *d_gw,
                             void *stream, lbm_obs *out);

/* Dynamic wetting (Sec. III.B, Fig. 7): advance n steps (a multiple of `every`) and record the
 * contact line on fluid row `row` at steps 0, every, 2 every, ..., n of this call, without any
 * host synchronisation. Sample k is written to d_series[2k] (leftmost rho_mid crossing where rho
 * rises, x linearly interpolated on the edge) and d_series[2k+1] (rightmost crossing where it
 * falls); both NaN when the row holds no liquid. d_series: caller-owned device memory of
 * count >= 2 (n/every + 1) doubles, written asynchronously on the context stream. The spreading
 * radius is (d_series[2k+1] - d_series[2k]) / 2. LBM_E_SIZE if count is too small. */
int lbm_record_contact_line(lbm_ctx *c, int64_t n, int32_t every, int32_t row, double *d_series,
                            size_t count);

/* Copy rho^n ([ny][nx], count >= nx*ny) or the pre-collision populations f^n ([9][ny][nx]) to
 * host memory. Synchronises the stream. Solid rows read 0. */
int lbm_read_rho(lbm_ctx *c, double *host, size_t count);
int lbm_read_f(lbm_ctx *c, double *host, size_t count);

/* Checkpoint: the full state (step counter and populations) as an opaque host blob of
 * lbm_state_size() bytes. Loading checks the blob's size and geometry (LBM_E_STATE). */
int lbm_state_size(const lbm_ctx *c, size_t *bytes);
int lbm_save_state(lbm_ctx *c, void *host, size_t bytes);
int lbm_load_state(lbm_ctx *c, const void *host, size_t bytes);

/* Replace the wall wettability pattern ([2][nx] host array, or [ny][nx] per node for a solid
 * mask; copied). */
int lbm_set_gw(lbm_ctx *c, const double *gw_host);

/* Kernel schedule of lbm_step:
 *   0      fused single pass (psi of the tile halo recomputed from the populations; 144
 *          algorithmic bytes per lattice update), tile 64x8;
 *   1      two passes (psi pass, then the force-collide-stream pass reading psi through LDS);
 *   2      (default) two time steps per launch (the first step's populations stay in LDS;
 *          72 bytes per lattice update), an odd remainder step runs fused; output tile 64x8,
 *          or the wide 32x4 workgroups (schedule 39) on lattices of at most 384 such tiles;
 *   16+t   fused with tile shape t (0..7: 64x4, 64x8, 64x16, 128x4, and the overlapped
 *          62-column tiles with 4, 6, 8, 14 rows);
 *   32+t   two steps per launch with output tile t (0..5: 64x8, 64x4, 128x4, 64x16, 32x8,
 *          32x4; 6, 7: 64x4 and 32x4 with one thread per first-step node and the halo ring on
 *          threads of its own, 768 and 448 per workgroup, for lattices too small to fill the
 *          GPU).
 * All schedules give bit-identical populations. A solid mask accepts every schedule but
 * 20..23 (LBM_E_INVAL). */
int lbm_set_schedule(lbm_ctx *c, int32_t schedule);

/* ---- Gradients of a wetting objective with respect to the wall wettability G_w ------------- */
/*
 * Objective on the state f^N after N steps (walls = 1 only; other geometries get LBM_E_INVAL):
 * with the phase fraction
 * phi = (rho - rho_v)/(rho_l - rho_v) over fluid nodes, the centroid height
 * y_c = sum phi (y - 1/2) / sum phi and the wetted length l_w = sum_x phi(x, 1),
 *     L = w_centroid * y_c + w_wet * l_w.
 * The gradient dL/dG_w (the G_w of every solid node of both walls, which enter the adhesion
 * forces Eqs. 10, 11, 14) is obtained by a hand-written adjoint of Eqs. (1)-(11), (14), the
 * pseudopotential and the halfway bounce-back, with checkpoint-every-K recomputation:
 *  1. lbm_forward_ckpt(c, N, K, ws, bytes) advances c by N steps and stores the state every K
 *     steps in the device workspace ws (>= lbm_adjoint_workspace_size() bytes, 256-aligned,
 *     caller-owned);
 *  2. lbm_loss() evaluates L on the current state (synchronises);
 *  3. lbm_backward(c, N, K, ws, bytes, w_centroid, w_wet, d_grad) must follow the matching
 *     lbm_forward_ckpt on the same context (LBM_E_STATE otherwise). It recomputes each segment of
 *     K steps from its checkpoint, runs the adjoint steps in reverse and writes dL/dG_w into the
 *     device array d_grad [2][nx] (row 0 bottom wall, row 1 top wall). Asynchronous on the
 *     context stream; the context's own state is left at step N. The recomputation of the next
 *     segment runs on a stream the context creates on first use (default priority, destroyed by
 *     lbm_destroy) while the current segment is reversed; the context stream waits for it, so
 *     all of the call's work is ordered before later work on the context stream.
 * Memory: ceil(N/K) + 2K states of 9 * ny * round_up(nx, 32) doubles, plus 26 planes.
 */
int lbm_adjoint_workspace_size(const lbm_params *p, int64_t nsteps, int32_t K, size_t *bytes);
int lbm_forward_ckpt(lbm_ctx *c, int64_t nsteps, int32_t K, void *d_ws, size_t bytes);
int lbm_loss(lbm_ctx *c, double w_centroid, double w_wet, double *L);
int lbm_backward(lbm_ctx *c, int64_t nsteps, int32_t K, void *d_ws, size_t bytes,
                 double w_centroid, double w_wet, double *d_grad_gw);

/* ---- Ensembles of uneven lattices -------------------------------------------------------- */
/*
 * `count` independent instances (each with its own lbm_params: lattice size, wall force, G_w,
 * viscosities ...) advanced together. All instances' tiles form one work-list, executed by one
 * launch per time step (schedule 0) or per two steps (schedule 2), replayed from captured
 * hipGraphs, or by one persistent launch for n steps (schedule 1: an occupancy-sized grid whose
 * workgroups take tiles from a ticket counter per XCD and advance them two steps at a time, with
 * a grid barrier between the two-step passes, and a per-step launch for an odd last step;
 * lbm_batch_step is then a single hipGraphLaunch; each wait at a barrier gives up after
 * LBM_PERSISTENT_SPIN_LIMIT polls, an environment variable read when the ensemble is created
 * (default 4,194,304), and ends the whole run through an abort flag that the next observables call
 * reports as LBM_E_HIP). The persistent grid fills the GPU: its workgroups must all be resident at
 * once, so a persistent run must not share the GPU with other kernels that hold compute units for
 * long (another persistent run included); if they do, its barriers time out and the run aborts as
 * above rather than hang. All run
 * the same per-tile arithmetic as lbm_step, so every instance evolves bit-for-bit as it would
 * alone.
 */
typedef struct {
    int32_t tile;         /* tile shape 0..4: 64x4, 64x8, 64x16, 128x4, 32x4 (the last's
                             two-step workgroups have one thread per first-step node: for
                             ensembles too small to fill the GPU) */
    int32_t reserved;     /* must be 0 */
    int32_t waves_per_cu; /* persistent schedule: workgroups per compute unit (0 = occupancy) */
    int32_t schedule;     /* 0 per-step launches, 1 persistent, 2 two steps per launch (output
                             tiles of the tile shape) */
} lbm_tune;

typedef struct lbm_batch lbm_batch;

/* Device workspace bytes for the ensemble (tune may be NULL: tile 1, per-step schedule). */
int lbm_batch_workspace_size(const lbm_params *p, int32_t count, const lbm_tune *tune,
                             size_t *bytes);
/* p[count]: parameters; gw_host[count] ([2][nx] each) and rho0_host[count] ([ny][nx] each):
 * host arrays, copied; d_ws: caller-owned device workspace (256-byte aligned). Solid masks are
 * rejected here (LBM_E_INVAL): use lbm_batch_create_masked. */
int lbm_batch_create(const lbm_params *p, int32_t count, const double *const *gw_host,
                     const double *const *rho0_host, const lbm_tune *tune, void *d_ws,
                     size_t bytes, void *hip_stream, lbm_batch **out);
/* An ensemble of solid-mask lattices (every p[i].walls = LBM_WALLS_MASK; see lbm_create_masked):
 * solid_host[count] ([ny][nx] bytes each), gw_host[count] ([ny][nx] G_w per node each),
 * rho0_host[count]; all copied. Every schedule of lbm_tune. */
int lbm_batch_create_masked(const lbm_params *p, int32_t count, const uint8_t *const *solid_host,
                            const double *const *gw_host, const double *const *rho0_host,
                            const lbm_tune *tune, void *d_ws, size_t bytes, void *hip_stream,
                            lbm_batch **out);
/* Advance every instance by n steps (asynchronous). */
int lbm_batch_step(lbm_batch *b, int64_t n);
/* Observables of every instance into out[count]; synchronises. LBM_E_HIP if a persistent run
 * was aborted by the grid-barrier time-out (workgroups not co-resident). */
int lbm_batch_observables(lbm_batch *b, lbm_obs *out);
/* Same with the contact plane of every instance given (y_wall[count]; see
 * lbm_observables_plane), or the default planes when y_wall is NULL. */
int lbm_batch_observables_plane(lbm_batch *b, const double *y_wall, lbm_obs *out);
/* Dynamic wetting for an ensemble (see lbm_record_contact_line): advance every instance n steps
 * (a multiple of every) and record the contact line of instance i on its fluid row rows[i] at
 * steps 0, every, ..., n of the call: sample k of instance i in d_series[2 (k count + i)] and
 * d_series[2 (k count + i) + 1]. d_series: device memory of >= 2 count (n/every + 1) doubles,
 * filled asynchronously on the ensemble's stream. */
int lbm_batch_record_contact_line(lbm_batch *b, int64_t n, int32_t every, const int32_t *rows,
                                  double *d_series, size_t count);
/* Gradients for a whole ensemble (every instance with walls = 1): the objective and the adjoint
 * of the single-lattice entry points above (lbm_loss, lbm_forward_ckpt, lbm_backward) for every
 * instance at once. The forward part advances the ensemble by nsteps with its own schedule and
 * stores every instance's state every K steps; the backward part recomputes each segment of all
 * instances with two-step launches over one work-list of 64 x 4 tiles and runs each reverse step
 * of all instances as one launch over the same work-list. Every instance's gradient is bit for bit
 * the one its lattice alone gets from lbm_backward.
 *   lbm_batch_adjoint_workspace_size: device bytes for (nsteps, K): per instance ceil(N/K) + K
 *     states and the adjoint buffers of lbm_adjoint_workspace_size, plus the tables;
 *   lbm_batch_forward_ckpt: d_ws caller-owned, 256-byte aligned, >= that size;
 *   lbm_batch_loss: L[count] host array (synchronises);
 *   lbm_batch_backward: must follow the matching lbm_batch_forward_ckpt (LBM_E_STATE otherwise);
 *     writes dL/dG_w of instance i ([2][nx_i], bottom then top wall) to the device array d_grad
 *     at offset sum_{j<i} 2 nx_j; asynchronous on the ensemble's stream.
 * LBM_E_INVAL when an instance has another geometry. */
int lbm_batch_adjoint_workspace_size(const lbm_batch *b, int64_t nsteps, int32_t K,
                                     size_t *bytes);
int lbm_batch_forward_ckpt(lbm_batch *b, int64_t nsteps, int32_t K, void *d_ws, size_t bytes);
int lbm_batch_loss(lbm_batch *b, double w_centroid, double w_wet, double *L);
int lbm_batch_backward(lbm_batch *b, int64_t nsteps, int32_t K, void *d_ws, size_t bytes,
                       double w_centroid, double w_wet, double *d_grad);
/* Pre-collision populations f^n of instance `index` ([9][ny][nx] host array). */
int lbm_batch_read_f(lbm_batch *b, int32_t index, double *host, size_t count);
/* State of instance `index` as a checkpoint blob (the format of lbm_save_state, loadable into
 * a single-instance context with the same parameters by lbm_load_state); synchronises. */
int lbm_batch_save_state(lbm_batch *b, int32_t index, void *host, size_t bytes);
int64_t lbm_batch_current_step(const lbm_batch *b);
/* The tune in use and the persistent grid size (workgroups). */
int lbm_batch_get_tune(const lbm_batch *b, lbm_tune *t, int32_t *grid);
/* Release an ensemble: waits for its queued work (graph replays included), then frees the
 * captured graphs and the host handle; the workspace may be freed once it returns. */
int lbm_batch_destroy(lbm_batch *b);
const char *lbm_batch_last_error(const lbm_batch *b);
/* Autotuner: times every tile shape x schedule (per-step launches, persistent at full and half
 * occupancy, two-step launches) for `steps` steps on this ensemble in the given workspace, in two
 * sweeps (each candidate counts with its faster run), and returns the fastest tune and its time
 * in milliseconds. */
int lbm_autotune(const lbm_params *p, int32_t count, const double *const *gw_host,
                 const double *const *rho0_host, void *d_ws, size_t bytes, void *hip_stream,
                 int32_t steps, lbm_tune *best, double *best_ms);

int64_t lbm_current_step(const lbm_ctx *c);

/* The device's FP64 square root and division as the step kernels compile them (the pseudo-
 * potential's square root and the velocity's division of Eq. 6 rely on them): for i < n,
 * d_sqrt[i] = sqrt(d_a[i]) and d_quot[i] = d_a[i] / d_b[i]. All four are device arrays of n
 * doubles, caller-owned; asynchronous on `stream`. For checking their rounding against the host's
 * correctly rounded operations. LBM_E_INVAL for null arrays (n > 0) or n > 2^36. */
int lbm_fp64_probe(const double *d_a, const double *d_b, double *d_sqrt, double *d_quot, size_t n,
                   void *stream);

/* Release a context (host memory only). Waits for the work queued on its stream first, so the
 * caller may free the workspace as soon as it returns; LBM_E_HIP if that wait failed (the
 * context is released all the same). */
int lbm_destroy(lbm_ctx *c);
const char *lbm_strerror(int code);
const char *lbm_last_error(const lbm_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
