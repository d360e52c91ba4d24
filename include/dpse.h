/*
 * dpse.h -- C ABI of the doubly-periodic spectral Ewald (DP-SE) solver for
 * MI355X (gfx950).
 *
 * The library computes, for N charges q_k at positions z_k in a slab
 * 0 < z < H that is periodic in x (period Lx) and y (period Ly), with
 * permittivity eps inside, eps_bottom below z = 0 and eps_top above z = H:
 *   - the energy U = 1/2 sum_k q_k phibar_k            (paper Sec. 2, eq. Ufinal),
 *   - the averaged potential phibar_k at each charge     (eq. pbar), and
 *   - the force F_k = q_k Ebar(z_k)                      (eq. fqE),
 * with the Poisson equation eps*Lap(phi) = -rho (eq. poiss) and the jump
 * conditions of eqs. cbc1-cbc4, with optional fixed charge densities on the
 * walls (eq. rho; dpse_plan_set_walls), whose wall integral then joins U as
 * in eq. Ufinal. The method is the paper's
 * Ewald split (Sec. 3.2) into a localized near field summed over pairs
 * (Sec. 4.2) and a smooth far field solved on a grid that is Fourier in x,y
 * and Chebyshev in z, with images of charges near the walls and a harmonic
 * correction for the rest of the image series (Sec. 4.3, algorithm of
 * Sec. 5.2.2 steps 1-7, per-mode boundary value solver of App. A).
 *
 * Units: a point charge q at distance r in a uniform medium has potential
 * q/(4 pi eps r). The charges and the wall charge densities together must
 * be exactly neutral (eq. elecneu).
 *
 * Conventions fixed by this library where the paper is silent:
 *   - g_w = 0 gives point charges; the self potential of each charge is
 *     removed as in Sec. 6.3, so phibar and U are finite;
 *   - support n_g = 2*ceil(4.3*g_t/h) grid cells unless given (Sec. 5.1);
 *   - z grid: Gauss-Lobatto Chebyshev nodes on [-3 H_E, H + 3 H_E] (Sec. 5.2.2);
 *   - gauge phi(0) = 0 (eq. phi00, Sec. 5.2.2) unless DPSE_GAUGE_NONE;
 *   - near field: pairs with minimal-image distance r < r_cut, one image of
 *     every charge per wall (Sec. 4.2, 5.2.2).
 *
 * Streams and ownership. All position, charge and output pointers are DEVICE
 * pointers owned by the caller (e.g. torch.Tensor.data_ptr() of float64 HIP
 * tensors). A plan from dpse_plan_create owns its workspace; a plan from
 * dpse_plan_create_unbound uses caller-owned device memory attached with
 * dpse_plan_bind (so that many plans can share one arena, one plan at a time
 * per stream). dpse_solve only enqueues work on
 * the plan's HIP stream and returns; the caller's buffers must stay valid
 * until that stream has passed the solve. A plan is not thread safe and must
 * not run two solves concurrently. Data-dependent errors (charge outside the
 * slab, non-neutral set, constraint violated) are detected on the device and
 * returned by the next dpse_sync; outputs of such a solve are undefined.
 */
#ifndef DPSE_H
#define DPSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (every entry point returns one; 0 is success). */
enum {
  DPSE_OK = 0,
  DPSE_EINVAL = 1,      /* invalid argument or parameters                        */
  DPSE_ENOMEM = 2,      /* device allocation failed                              */
  DPSE_EHIP = 3,        /* a HIP runtime call failed                             */
  DPSE_ENONNEUTRAL = 4, /* |sum q + int sigma| > 1e-12 (sum |q| + int |sigma|)  (device-detected) */
  DPSE_EOUTSIDE = 5,    /* a charge with z outside (n_sigma g_w, H - n_sigma g_w), or a non-finite coordinate (device-detected) */
  DPSE_ECONSTRAINT = 6, /* r_cut >= H + h_min or 2 H_E >= H + h_min, h_min the smallest distance of a charge to a wall (Sec. 4.2, 5.3; device-detected) */
  DPSE_ETOOMANY = 7,    /* n larger than the plan's max_n                        */
  DPSE_ESCRATCH = 8     /* the plan's workspace exceeds the static scratch buffer of dpse_solve_static */
};

/* Precision of the grid stages. */
enum {
  DPSE_FP64 = 0,  /* every stage in FP64                                          */
  DPSE_MIXED = 1  /* spreading, x,y FFTs, interpolation, near field in FP32 with FP32
                     accumulation; z transforms, per-mode solves, harmonic
                     correction, k = 0 mode and all per-charge sums in FP64    */
};

/* Flags (bitwise or). */
enum {
  DPSE_GAUGE_NONE = 1,  /* skip the phi(0) = 0 gauge constant (U and F unaffected for neutral sets) */
  DPSE_KMAX_GT = 2,     /* cap the harmonic correction at |k| <= min(pi/h, 4.2/g_t) instead of pi/h */
  DPSE_UNIFORM_FAST = 4, /* equal permittivities (eps_bottom == eps == eps_top, else DPSE_EINVAL):
                           the free-space solve of Sec. 3.1.1 on the Chebyshev domain [-H_E, H + H_E],
                           with no wall group, images or harmonic correction, and the k = 0 slope
                           that cancels the field outside the (neutral) sources; about half the
                           z nodes of the general solver for the same accuracy */
  DPSE_ONE_JUMP = 8,    /* a jump at exactly one wall (eps_top == eps != eps_bottom or the
                           reverse, else DPSE_EINVAL; not with DPSE_UNIFORM_FAST): every charge
                           is imaged across that wall (Sec. 4 opening: for one interface the
                           image construction is exact) and the free-space solve of
                           DPSE_UNIFORM_FAST runs on the span of charges and images,
                           [-H - H_E, H + H_E] (bottom) or [-H_E, 2H + H_E] (top); no wall
                           group or correction. Shorter than the general domain when
                           H < 4 H_E; no wall charges */
  DPSE_TRIPLY = 16,     /* triply periodic variant (Sec. 7 and its performance comparison): the box
                           is periodic in z too, with period H (the permittivities must be equal,
                           and the walls play no part); a uniform z grid of Nz nodes (a power of two
                           in [32, 1024]), the far field solved by Fourier transforms in all three
                           directions (psi^ = f^ / (eps |k|^2), psi^(0) = 0), the near field over
                           minimal images in x, y and z; no gauge constant (the k = 0 mode is zero);
                           needs H >= 4 H_E and r_cut < H / 2; not with the other solver flags */
  DPSE_DETERMINISTIC = 32 /* bitwise-reproducible solves: the same inputs give the same output bits
                           on every run, alone or beside other work on the device. No floating-point
                           atomics: the spreading and near-field cell lists are put in a fixed order
                           inside every bin and cell after the counting sorts, spreading runs in its
                           gather form with one block per tile, and interpolation with one wavefront
                           per charge (a fixed-order sum and a plain store); every other reduction
                           already has a fixed order. Overrides the tuned shapes of spreading and
                           interpolation (dpse_plan_autotune and dpse_plan_set_tiles leave them to
                           this rule). Slower than the default path; results agree with it to
                           rounding */
};

/* Parameters of one slab system. Lengths share one unit. */
typedef struct {
  double Lx, Ly, H;                 /* periods in x,y; slab height; > 0                      */
  double eps, eps_bottom, eps_top;  /* permittivities; > 0                                   */
  double xi;                        /* Ewald splitting parameter (eq. gamreal); > 0          */
  double g_w;                       /* Gaussian charge width (eq. gcharge); >= 0             */
  int32_t Nx, Ny, Nz;               /* grid; Nx, Ny powers of two in [32, 1024]; Nz - 1 a power of two in [32, 1024] (Nz itself with DPSE_TRIPLY); Lx/Nx == Ly/Ny */
  int32_t support;                  /* n_g, even, <= 32; 0 = 2*ceil(4.3*g_t/h)               */
  double r_cut;                     /* near cutoff, 0 < r_cut < min(Lx, Ly)/2; 0 = derive from delta (eq. rnf) */
  double delta;                     /* tolerance used when r_cut == 0 (default 1e-4 if 0)    */
  int32_t precision;                /* DPSE_FP64 or DPSE_MIXED                               */
  int32_t flags;                    /* DPSE_GAUGE_NONE | DPSE_KMAX_GT | DPSE_UNIFORM_FAST | DPSE_ONE_JUMP | DPSE_TRIPLY
                                       | DPSE_DETERMINISTIC */
} dpse_params;

/* Derived quantities of a plan (Sec. 3.2 eq. gt, Sec. 5.1 eq. He, Sec. 5.2.2). */
typedef struct {
  double h;            /* grid spacing in x and y                                 */
  double g_t;          /* std of the spreading Gaussian S-bar                     */
  double H_E;          /* support radius n_g h / 2                                */
  double n_sigma;      /* H_E / g_t                                               */
  double z_lo, z_hi;   /* Chebyshev domain ([-3 H_E, H + 3 H_E] with two jumps)   */
  double r_cut;        /* near cutoff actually used                              */
  double xi_e;         /* (4 g_w^2 + xi^-2)^(-1/2)                                */
  int32_t support;     /* n_g                                                      */
  int32_t n_modes;     /* Ny (Nx/2 + 1) transverse modes                          */
  int64_t workspace_bytes; /* device memory of one solve's workspace (0 from dpse_derive) */
  int64_t max_n;       /* charges per solve the plan accepts (0 from dpse_derive)  */
  int64_t table_bytes; /* device memory of the plan's resident tables, including the
                          factorised per-mode solver operators (0 from dpse_derive) */
} dpse_info;

typedef struct dpse_plan dpse_plan;

/* Validates params and fills info without touching the GPU (host only).
 * Returns DPSE_EINVAL (with info untouched) for invalid parameters. */
int dpse_derive(const dpse_params* params, dpse_info* info);

/* Creates a plan for up to max_n charges per solve on the HIP stream `stream`
 * (a hipStream_t; NULL = the null stream) of the current device. Allocates the
 * workspace and uploads the plan tables (nodes, quadrature weights, wave
 * numbers) and factorises the per-mode boundary value operators of App. A
 * (their elimination multipliers depend on |k| only; a kernel on a private
 * stream, waited for). *out receives the plan. */
int dpse_plan_create(const dpse_params* params, int64_t max_n, void* stream, dpse_plan** out);

/* Device bytes of the workspace of one solve of up to max_n charges with
 * these parameters (host only; the same figure as dpse_info.workspace_bytes). */
int dpse_workspace_size(const dpse_params* params, int64_t max_n, int64_t* bytes);

/* Creates a plan like dpse_plan_create but allocates only its tables (a few
 * KB to MB: nodes, weights, twiddles, per-mode solver coefficients) and no
 * workspace. Before its first solve the caller attaches a workspace with
 * dpse_plan_bind; entry points that need one return DPSE_EINVAL until then. */
int dpse_plan_create_unbound(const dpse_params* params, int64_t max_n, dpse_plan** out);

/* Attaches caller-owned device memory `workspace` (256-byte aligned, at
 * least dpse_workspace_size bytes; the caller keeps ownership and frees it
 * after the plan's last solve has finished) and the HIP stream `stream` to a
 * plan from dpse_plan_create_unbound. May be called again to move the plan to
 * other memory or another stream; the workspace holds no state between
 * solves except the device status of dpse_sync, which binding clears (with a
 * kernel on `stream`, ordered after the work already queued there). Plans that
 * share a workspace must run on one stream, or the caller orders them; they
 * share one status word (at the start of the workspace), which dpse_sync on
 * any of them reports and clears.
 * DPSE_EINVAL for a plan that owns its workspace, a null or misaligned
 * pointer, or too few bytes. */
int dpse_plan_bind(dpse_plan* plan, void* workspace, int64_t bytes, void* stream);

/* Copies the derived quantities of a plan into *info. */
int dpse_plan_info(const dpse_plan* plan, dpse_info* info);

/* Fixed charge densities sigma_b on the bottom wall (z = 0) and sigma_t on
 * the top wall (z = H) of a plan (Sec. 2 eq. rho and the jump conditions
 * cbc2, cbc4). Each solve then adds them to the displacement mismatches of
 * the harmonic correction (Sec. 4.3.3 eqs. mm2, mm4) and to the slope of the
 * k = 0 mode (Sec. 4.3.4 eqs. ai1, ai2), and the energy gains the wall
 * integral of eq. Ufinal, 1/2 int (sigma_b phi(x,y,0) + sigma_t phi(x,y,H)),
 * taken by reciprocity: with phi_s the potential of the walls alone (their
 * correction, harmonic in the slab) and B the gauge constant,
 *   int sigma phi = sum_k q_k phi_s(z_k) + int sigma phi_s + B int sigma,
 * the first sum from the S-bar averages of phi_s at the charges, the second
 * from the wall modes (both FP64). Neutrality becomes sum q + int sigma = 0.
 *   sigma_b, sigma_t  device, [Ny][Nx] float64 (x fastest): the densities at
 *                     the grid points (i h, j h); NULL = no charge on that
 *                     wall; both NULL removes the wall charges.
 * The densities must be resolved by the grid (the correction keeps only the
 * modes the plan corrects). The call copies what it needs (the caller's
 * buffers may be reused once the plan's stream has passed it), enqueues its
 * kernels on the plan's stream and uses the workspace, so the plan must be
 * bound; the wall data (the transforms and the FP32 or FP64 grid of phi_s,
 * Nz Ny Nx reals) is allocated once and kept with the plan. Captured graphs
 * of dpse_solve_graph are re-captured; batch graphs keep the wall state of
 * their creation. DPSE_EINVAL for an unbound plan or a DPSE_UNIFORM_FAST plan
 * (it has no correction), DPSE_ENOMEM, DPSE_EHIP. */
int dpse_plan_set_walls(dpse_plan* plan, const double* sigma_b, const double* sigma_t);

/* Enqueues one solve (Sec. 5.2.2 steps 1-7 plus the near field). The near
 * field needs only its cell list: that list and the near field run on a
 * stream private to the plan, forked from the plan's stream once the forward
 * transforms are queued and joined back before the gauge constant,
 * concurrently with the column solve and the later far-field stages. */
/* Arguments of dpse_solve:
 *   n      number of charges, 1 <= n <= max_n;
 *   pos    device, n x 3 row-major float64 (x, y, z); x, y are taken modulo Lx, Ly;
 *   q      device, n float64 charges;
 *   energy device, 1 float64, or NULL;
 *   phi    device, n float64 averaged potentials, or NULL;
 *   force  device, n x 3 row-major float64 forces, or NULL.
 * Outputs are in the caller's charge order. Host-detectable errors return
 * immediately (DPSE_EINVAL, DPSE_ETOOMANY); data errors appear at dpse_sync. */
int dpse_solve(dpse_plan* plan, int64_t n, const double* pos, const double* q,
               double* energy, double* phi, double* force);

/* The solve of dpse_solve as one HIP graph launch. The first call (and any
 * call whose n, pointers, workspace or stream differ from the previous one)
 * captures the solve's kernels into a graph (no allocation or memset node:
 * buffers are cleared by kernels) and instantiates it; later calls with the
 * same arguments only launch it, which removes the per-kernel launch cost for
 * small systems. Stage timing is not recorded for graph solves, and the near
 * field runs on the capturing stream instead of the plan's side stream. Same
 * arguments, results and errors as dpse_solve. */
int dpse_solve_graph(dpse_plan* plan, int64_t n, const double* pos, const double* q,
                     double* energy, double* phi, double* force);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The solve of
 * dpse_solve (same arguments, results and device errors) with its workspace
 * in a static device array of the library, 64 MiB per device, held from the
 * library's first use on that device until the process ends. The call
 * allocates nothing (no hipMalloc, hipFree, event or stream creation) and
 * enqueues its kernels on `stream` (a hipStream_t; NULL = the null stream).
 *   plan   from dpse_plan_create_unbound (its tables were allocated when it
 *          was created); it stays bound to the static array and `stream`
 *          after the call (dpse_sync, dpse_solve_near and dpse_debug_copy then
 *          read the array; dpse_plan_bind moves it elsewhere);
 *   n, pos, q, energy, phi, force  as for dpse_solve; per-stage timing is
 *          not recorded.
 * Every call on a device shares that device's array, whose contents stay
 * from the last call: the call clears the status word with a kernel and every
 * other buffer is rewritten by the solve's own kernels. Calls that overlap on
 * one device (other streams, other threads, other plans) race on the array;
 * the caller orders them. DPSE_ESCRATCH when dpse_info.workspace_bytes
 * exceeds 64 MiB (about 52 bytes per grid point in DPSE_MIXED, 104 in
 * DPSE_FP64, plus about 300 per charge of max_n: the 32 x 32 x 33 grid with
 * 64 charges takes 3.5 MiB in FP64, a 128 x 128 x 65 grid with 3.5 * 10^4
 * charges 63.9 MiB in DPSE_MIXED), DPSE_EINVAL for a plan that
 * owns its workspace or bad arguments, DPSE_ETOOMANY. */
int dpse_solve_static(dpse_plan* plan, void* stream, int64_t n, const double* pos, const double* q,
                      double* energy, double* phi, double* force);

/* Reuse of the far field between time steps (the paper's closing remark on
 * reusing far-field work between Brownian-dynamics steps, Sec. 8): the near
 * field (Sec. 4.2) of the charges at pos, plus each charge's far-field
 * average (potential and field) and the gauge constant of the plan's last
 * full solve (dpse_solve, dpse_solve_graph or a batch), held fixed:
 *   phibar_k = phibar^f_k(last) + phibar^n_k(pos) + B(last) - self term,
 *   F_k = q_k (Ebar^f_k(last) + Ebar^n_k(pos)), U = 1/2 sum q phibar plus the
 *   wall terms of the last full solve.
 * Costs the validation, the binning, the near field and the outputs, about a
 * quarter of a full solve. The last full solve must have had the same n and
 * the same charges q in the same order (the caller's contract). The far-field
 * averages live in the workspace: the library keeps, per workspace, which
 * plan's full solve last wrote them (a full solve, a replay of
 * dpse_solve_graph or a launch of a batch graph holding the plan), and binding
 * or dpse_plan_set_walls invalidates them. Same arguments, outputs and device
 * errors as dpse_solve; DPSE_EINVAL without a full solve of this n to reuse,
 * or when another plan has solved in the workspace (a shared arena) since. */
int dpse_solve_near(dpse_plan* plan, int64_t n, const double* pos, const double* q,
                    double* energy, double* phi, double* force);

/* One Brownian-dynamics step of the non-Markovian Euler-Maruyama scheme of
 * Leimkuhler and Matthews that the paper integrates with (Sec. 7, eq.
 * leimkuhler), for forces computed by a solve:
 *   pos_out = pos + mu_dt force + noise (w_prev + w_next),  noise = sqrt(kT mu dt / 2),
 * all device, n x 3 row-major float64 (w_prev, w_next standard normal draws of
 * the caller; pos_out must not alias pos, so that a rejected step leaves pos
 * as it was). *escaped (device int32) receives the number of charges whose
 * new height is not strictly inside the admissible range of dpse_solve
 * (n_sigma g_w, H - n_sigma g_w); the paper discards such a step and retries
 * it with new noise. x and y are left unwrapped (the solve takes them modulo
 * the periods). Enqueued on the plan's stream. */
int dpse_bd_step(dpse_plan* plan, int64_t n, const double* pos, const double* force, const double* w_prev,
                 const double* w_next, double mu_dt, double noise, double* pos_out, int32_t* escaped);

/* Enqueues n_sys independent solves (one per plan, each with its own sizes and
 * parameters) as one batch. Array arguments have n_sys entries with the
 * meaning of dpse_solve's. Plans may share a stream; the batch is ordered on
 * the stream of plans[0], and every other plan's stream waits for it. */
int dpse_solve_batch(int n_sys, dpse_plan* const* plans, const int64_t* n,
                     const double* const* pos, const double* const* q,
                     double* const* energy, double* const* phi, double* const* force);

/* A batch of solves captured into one HIP graph: one launch runs every
 * system of the batch (the work of dpse_solve_batch). System i runs on branch
 * branch[i] (0 <= branch[i] < n_branches <= 64; NULL = i mod n_branches);
 * systems of one branch run in the given order, different branches may run
 * concurrently, so plans bound to one workspace must share a branch. The
 * graph records the pointers and sizes given here: relaunching it solves
 * again with whatever those buffers then hold. The plans must stay alive
 * and bound to the same workspaces while the graph exists. Stage timing is
 * not recorded. dpse_graph_launch enqueues the whole batch on `stream`;
 * device-side statuses go to each plan's workspace (dpse_sync). */
typedef struct dpse_graph dpse_graph;
int dpse_batch_graph_create(int n_sys, dpse_plan* const* plans, const int64_t* n,
                            const double* const* pos, const double* const* q,
                            double* const* energy, double* const* phi, double* const* force,
                            const int32_t* branch, int n_branches, dpse_graph** out);
int dpse_graph_launch(dpse_graph* graph, void* stream);
int dpse_graph_destroy(dpse_graph* graph);

/* Launch shapes picked per grid. Spreading and interpolation work on LDS
 * tiles of T x T grid columns by P Chebyshev nodes; the column kernel on
 * blocks of KE / (2(Nz-1)) modes (KE complex LDS elements per buffer). The
 * fastest shapes depend on the grid, the support and the charge density.
 * dpse_plan_autotune runs one solve of the given charges (outputs discarded),
 * then times every applicable candidate of each tuned stage `reps` times with
 * HIP events on the plan's stream, keeps the fastest in the plan, writes the
 * chosen candidate of stage s (0 spreading, 1 interpolation, 2 column) to
 * choice[s] if choice is not NULL (DPSE_NUM_TUNED entries), and the mean
 * milliseconds of candidate i of stage s to ms[DPSE_MAX_CANDIDATES s + i] (-1
 * where a candidate does not apply) if ms is not NULL (DPSE_MAX_CANDIDATES *
 * DPSE_NUM_TUNED entries). Synchronous;
 * returns the device status of the solve like dpse_sync. dpse_plan_set_tiles
 * applies stored choices (-1 = the default rule) to a plan of the same grid;
 * DPSE_EINVAL if a choice does not apply. Results depend on the choice only
 * through rounding (the order of floating-point sums). */
enum { DPSE_NUM_TUNED = 3, DPSE_MAX_CANDIDATES = 16 };
int dpse_plan_autotune(dpse_plan* plan, int64_t n, const double* pos, const double* q, int reps,
                       int32_t* choice, double* ms);
int dpse_plan_set_tiles(dpse_plan* plan, const int32_t* choice);

/* Waits for the plan's stream and returns the device-side status of the
 * solves enqueued since the previous dpse_sync (DPSE_OK, DPSE_ENONNEUTRAL,
 * DPSE_EOUTSIDE or DPSE_ECONSTRAINT), clearing it. */
int dpse_sync(dpse_plan* plan);

/* Frees the plan and its workspace (waits for its stream first). */
int dpse_plan_destroy(dpse_plan* plan);

/* Static description of a status code. */
const char* dpse_status_string(int status);

/* Stage outputs kept in the workspace after a solve, for per-stage checks.
 * dpse_debug_copy waits for the plan's stream and copies stage `which` into
 * host memory `dst` (at most `bytes` bytes); *elem_bytes receives the size of
 * one real (8 or 4) and *count the number of reals copied. Layouts:
 *   DPSE_STAGE_F_I    spread grid of all charges and images, [Nz][Ny][Nx]
 *   DPSE_STAGE_F_O    spread grid of the wall-band charges, [Nz][Ny][Nx] (zero outside the bands)
 *   DPSE_STAGE_FH_I   x,y transform of F_I, complex [Nz][Ny][Nx/2+1] (re, im interleaved)
 *   DPSE_STAGE_PSI    potential at the nodes per mode, complex [Nz][Ny][Nx/2+1]
 *   DPSE_STAGE_PSIZ   z-derivative of it, complex [Nz][Ny][Nx/2+1]
 *   DPSE_STAGE_GRIDS  phi, Ex, Ey, Ez on the grid, [Nz][Ny][Nx][4]
 *   DPSE_STAGE_FAR    far-field averages at the charges (phi, Ex, Ey, Ez), [n][4], caller order
 *   DPSE_STAGE_NEAR   near-field sums at the charges (phi, Ex, Ey, Ez), [n][4], caller order
 *   DPSE_STAGE_SCALARS (B_i, A_i, far part at the origin, near part at the origin), FP64
 *   DPSE_STAGE_WALL_HAT   x,y transforms of sigma_b then sigma_t, complex [2][Ny][Nx/2+1], FP64
 *   DPSE_STAGE_WALL_PHI   potential of the wall charges alone on the grid, [Nz][Ny][Nx]
 *   DPSE_STAGE_WALL_SCALARS (int sigma, int |sigma|, int sigma phi_s, k = 0 slope of phi_s), FP64
 *   DPSE_STAGE_FH_O   x,y transform of F_O, complex [Nz][Ny][Nx/2+1] (zero outside the bands)
 * (the wall entries after dpse_plan_set_walls) */
enum {
  DPSE_STAGE_F_I = 0, DPSE_STAGE_F_O = 1, DPSE_STAGE_FH_I = 2, DPSE_STAGE_PSI = 3,
  DPSE_STAGE_PSIZ = 4, DPSE_STAGE_GRIDS = 5, DPSE_STAGE_FAR = 6, DPSE_STAGE_NEAR = 7,
  DPSE_STAGE_SCALARS = 8, DPSE_STAGE_WALL_HAT = 9, DPSE_STAGE_WALL_PHI = 10, DPSE_STAGE_WALL_SCALARS = 11,
  DPSE_STAGE_FH_O = 12
};
int dpse_debug_copy(dpse_plan* plan, int which, void* dst, int64_t bytes,
                    int32_t* elem_bytes, int64_t* count);

/* Per-stage device timing. The paper reports the time of each stage of a
 * solve (Sec. 7.4: correction, spreading, near field, interpolation,
 * transforms, boundary value solves). With timing on, every solve records HIP
 * events between its stages on the plan's stream (no synchronization is
 * added). dpse_stage_times waits for the stream, writes the mean duration in
 * milliseconds of each stage over the solves recorded since the previous call
 * into ms[0 .. min(max_stages, DPSE_NUM_STAGES)), sets *n_solves, and clears
 * the record. Stage names come from dpse_stage_name. */
enum { DPSE_NUM_STAGES = 10 };
int dpse_set_timing(dpse_plan* plan, int enable);
int dpse_stage_times(dpse_plan* plan, double* ms, int max_stages, int* n_solves);
const char* dpse_stage_name(int stage);

#ifdef __cplusplus
}
#endif

#endif /* DPSE_H */
