// Internal declarations of the DP-SE library: plan constants passed to every
// kernel, the plan/workspace layout, and the launch wrappers of each stage.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "dpse.h"

namespace dpse {

constexpr double kPi = 3.14159265358979323846;

// Plan constants, passed by value as a kernel argument.
struct Geom {
  double Lx, Ly, H, eps, eps_b, eps_t, xi, g_w;
  double h, inv_h, g_t, H_E, za, zb, zc, zR;
  double gamma_b, gamma_t, tau_b, tau_t, xi_e, r_cut;
  double sbar_norm;  // (2 pi g_t^2)^(-3/2)
  double inv2g2;     // 1/(2 g_t^2)
  double zmin_ok, zmax_ok;  // admissible charge heights (exclusive bounds)
  int Nx, Ny, Nz, nkx, ng, flags;
  // particle bins used by spreading and interpolation
  int B;                 // bin width in grid cells (x and y)
  int nbx, nby, nzb;     // bins in x, y; z buckets
  double zb_lo, zb_w;    // z bucket origin and width
  // near-field cell list
  int ncx, ncy, ncz;
  double cwx, cwy, cwz;
  // wall bands of the psi_o* solve, where the spread of the wall group can be
  // non-zero: nodes [top_lo, top_end) (H - 3 H_E < z <= H + H_E) and
  // [bot_begin, bot_end) (-H_E <= z < 3 H_E); the nodes descend with the index
  int top_lo, top_end, bot_begin, bot_end;
};

// Whether node c lies in a wall band (the wall-group grid is zero elsewhere).
__host__ __device__ inline bool in_band(const Geom& g, int c) {
  return (c >= g.top_lo && c < g.top_end) || (c >= g.bot_begin && c < g.bot_end);
}

// Whether nodes [c0, c1) meet a wall band.
__host__ __device__ inline bool meets_band(const Geom& g, int c0, int c1) {
  return (c0 < g.top_end && c1 > g.top_lo) || (c0 < g.bot_end && c1 > g.bot_begin);
}

// One particle record: position and strength.
struct Part {
  double x, y, z, q;
};

// Group of an extended particle (charge or image), stored in meta & 3.
enum { GRP_WALL = 0, GRP_INNER = 1, GRP_IMAGE = 2 };

// Layout of Tables::ctab.
constexpr int kCtabRows = 4;   // a_n, b_n, c_n, rhs scale
constexpr int kNumFun = 10;    // S1, S2, S3, S4, V0, VH, D0, DH, Ea, Eb
enum { FUN_S1 = 0, FUN_S2, FUN_S3, FUN_S4, FUN_V0, FUN_VH, FUN_D0, FUN_DH, FUN_EA, FUN_EB };

// Launch shapes.
constexpr int kBin = 16;      // particle bin width (grid cells)
constexpr int kMaxSupport = 32;  // n_g <= the tile width (one contiguous window run per tile)

template <typename R>
struct Cplx;
template <>
struct Cplx<double> { using T = double2; };
template <>
struct Cplx<float> { using T = float2; };

struct Workspace {
  // particles
  Part* ext = nullptr;        // [3 max_n] charges then images
  int* ext_meta = nullptr;    // group | (original index << 2)
  Part* srt = nullptr;        // sorted by (bin, z bucket)
  int* srt_meta = nullptr;
  int* bin_cnt = nullptr;     // [nkeys + 1]
  int* bin_off = nullptr;     // [nkeys + 1]
  int* bin_cur = nullptr;     // [nkeys]
  int* n_img = nullptr;       // [1]
  // near-field cell list over the charges
  Part* nsrt = nullptr;       // [max_n]
  int* nsrt_idx = nullptr;    // original index
  int* cell_cnt = nullptr;
  int* cell_off = nullptr;
  int* cell_cur = nullptr;
  // grids (R = double or float, C = complex of R)
  void* f_i = nullptr;   // R [Nz][Ny][Nx]
  void* f_o = nullptr;   // R [Nz][Ny][Nx], band planes only
  void* fx_i = nullptr;  // C [Nz][Ny][nkx]
  void* fx_o = nullptr;  // C [Nz][Ny][nkx], band planes only
  void* psi = nullptr;   // C [Nz][Ny][nkx]
  void* psiz = nullptr;  // C
  void* p0 = nullptr;    // C inverse y-pass outputs
  void* py = nullptr;    // C
  void* pz = nullptr;    // C
  void* u4 = nullptr;    // R [Nz][Ny][Nx][4]
  // per-charge accumulators (caller order)
  double4* far4 = nullptr;
  double4* near4 = nullptr;
  // scalars: 0 sum q, 1 sum |q|, 2 B_i, 3 A_i, 4 far0, 5 near0, 6 energy scratch
  double* scal = nullptr;
  double* partials = nullptr;  // block partial sums
  double* qpart = nullptr;     // per-block sums of q and |q| of the prep kernel, [2][ceil(max_n / 256)]
  // block sums and their offsets of the multi-block counting-sort scans
  // (bins on the plan's stream, cells on the side stream), [3 (nb + 1)] each
  int* scan_bin = nullptr;
  int* scan_cell = nullptr;
  int* status = nullptr;
};

struct Tables {
  double* z = nullptr;      // nodes [Nz]
  double* wq = nullptr;     // h^2 * Clenshaw-Curtis weight [Nz]
  double* T0 = nullptr;     // T_n(s(0)) [Nz]
  double* TH = nullptr;     // T_n(s(H))
  double* dT0 = nullptr;    // T_n'(s(0)) / R
  double* dTH = nullptr;    // T_n'(s(H)) / R
  double2* twx = nullptr;   // exp(-2 pi i k/Nx), k < Nx/2
  double2* twy = nullptr;   // exp(-2 pi i k/Ny)
  double2* twz = nullptr;   // exp(-2 pi i k/(2(Nz-1)))
  // per-mode solver tables, [kCtabRows * Nz + kNumFun * (Nz + 2)] doubles:
  // chain coefficients a_n, b_n, c_n, the right-hand-side scale of each
  // Chebyshev coefficient, then weight vectors of the linear functionals
  // (on y''_0..y''_{N-1}, y_0, y'_0; see k_column.hip)
  double* ctab = nullptr;
  float2* twx_f = nullptr;
  float2* twy_f = nullptr;
  // factorised per-mode chains: elimination multipliers, [Nz][Ny (Nx/2+1)]
  // (chain-major rows, see k_pivots in k_column.hip)
  double* cpiv = nullptr;
  // the linear functionals S1..DH of each mode's homogeneous chain solutions
  // (even chain y_0 = 1, odd chain y'_0 = 1), [Ny (Nx/2+1)][2][8] (scan kernel)
  double* hfun = nullptr;
};

// Fixed wall charge densities (dpse_plan_set_walls), one allocation per plan.
struct Walls {
  double* stage = nullptr;   // sigma_b then sigma_t at the grid points, [2][Ny][Nx]
  double2* hat = nullptr;    // their x,y transforms, [2][Ny][nkx] (fft_xy normalisation)
  void* phis = nullptr;      // R [Nz][Ny][Nx]: potential of the walls alone at the nodes
  double* scal = nullptr;    // 0 int sigma, 1 int |sigma|, 2 int sigma phi_s, 3 k = 0 slope A_s
  double* part = nullptr;    // block partials of the wall term in the interpolation
};

}  // namespace dpse

struct dpse_plan {
  dpse_params prm;
  dpse_info info;
  dpse::Geom g;
  dpse::Tables t;
  dpse::Workspace w;
  dpse::Walls walls;
  bool walls_on = false;               // wall charges set (dpse_plan_set_walls)
  int walls_version = 0;               // bumped by every dpse_plan_set_walls
  // where the solve being enqueued leaves the partials of sum q phi_s-bar
  // (the interpolation's gather shapes, else the per-charge kernel), or null
  double* wall_part = nullptr;
  int wall_nparts = 0;
  // charges of the last full solve whose far-field averages (far4) and gauge
  // constant (scal[2]) are still in the workspace, for dpse_solve_near; 0 = none
  int64_t far_n = 0;
  // identity of the plan and number of its full solves: the arena's owner
  // record (plan.cpp) names the plan and solve whose far field it holds
  uint64_t uid = 0;
  uint64_t full_solves = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int64_t max_n = 0;
  int64_t last_n = 0;
  int nkeys = 0;
  int ncells = 0;
  int npartials = 0;
  std::vector<void*> allocs;
  bool bound = false;                  // a workspace is attached
  bool owns_workspace = false;
  hipGraphExec_t graph_exec = nullptr; // captured solve (dpse_solve_graph)
  const void* graph_sig[8] = {};
  hipStream_t graph_stream = nullptr;
  // tile shapes of spreading and interpolation: index into the candidate
  // lists of k_grid.hip, or -1 for the default rule (dpse_plan_autotune)
  int spread_cfg = -1;
  int interp_cfg = -1;
  int column_cfg = -1;   // modes per column block (kColumnKE of k_column.hip)
  // the near field runs on `side`, forked from and joined back into `stream`
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  bool capturing = false;  // inside a graph capture: no fork
  // per-stage timing: one row of 2 DPSE_NUM_STAGES events (start, end) per recorded solve
  bool timing = false;
  std::vector<hipEvent_t> events;
  int timed_solves = 0;
};

namespace dpse {

// Stage launchers (each enqueues on plan->stream). R = double or float.
hipError_t launch_prep(dpse_plan* p, int64_t n, const double* pos, const double* q);
hipError_t launch_bin(dpse_plan* p, int64_t n);        // both of:
hipError_t launch_bin_grid(dpse_plan* p, int64_t n);   // bins of spreading and interpolation
hipError_t launch_bin_cells(dpse_plan* p, int64_t n);  // cell list of the near field
template <typename R> hipError_t launch_spread(dpse_plan* p);
template <typename R> hipError_t launch_fft_forward(dpse_plan* p);
template <typename R> hipError_t launch_column(dpse_plan* p);
template <typename R> hipError_t launch_fft_inverse(dpse_plan* p);
template <typename R> hipError_t launch_interp(dpse_plan* p, int64_t n);
template <typename R> hipError_t launch_near(dpse_plan* p, int64_t n);
template <typename R> hipError_t launch_gauge_far(dpse_plan* p);
hipError_t launch_near_origin(dpse_plan* p, int64_t n);
hipError_t launch_finalize(dpse_plan* p, int64_t n, const double* q, double* energy,
                           double* phi, double* force, bool gauge);
hipError_t launch_bd_step(dpse_plan* p, int64_t n, const double* pos, const double* force, const double* w_prev,
                          const double* w_next, double mu_dt, double noise, double* pos_out, int* escaped);

// Tile-shape candidates of spreading (stage 0) and interpolation (stage 1):
// count, shape of candidate i (x,y tile width T and z nodes per block P), and
// whether it applies to the plan's grid.
int tile_candidates(int stage);
void tile_shape(int stage, int i, int* T, int* P);
bool tile_valid(const Geom& g, int stage, int i, bool fp64);
// Column-kernel block sizes (complex LDS elements per buffer).
int column_candidates();
// Plan-time factorisation of the per-mode chains into Tables::cpiv.
hipError_t launch_pivots(dpse_plan* p, hipStream_t s);
int column_block(int i);
bool column_valid(const Geom& g, int i);

// Wall charges: the x,y transforms of the staged densities (FP64), the
// potential of the walls alone at the nodes into the workspace's psi/psiz
// (the inverse transforms then give its grid), the wall scalars, the copy of
// that grid into Walls::phis, and the per-solve sum of q phi_s at the charges.
hipError_t launch_wall_transforms(dpse_plan* p);
template <typename R> hipError_t launch_wall_modes(dpse_plan* p);
template <typename R> hipError_t launch_wall_keep_phi(dpse_plan* p);
template <typename R> hipError_t launch_wall_energy(dpse_plan* p, int64_t n);
int wall_energy_blocks(const dpse_plan* p, int64_t n);
int gather_splits(const dpse_plan* p, int blocks, int T, int P);

// Sets kernel attributes once (before any stream capture).
hipError_t prepare_kernels();

// Workgroups are handed to the 8 XCDs in turn (workgroup b to XCD b mod 8)
// and every XCD has an L2 of its own. Where neighbouring workgroups share
// 128-byte lines (mode blocks of the column solve, kx column blocks of the y
// transforms, whose rows of nkx complex values are not line-aligned), the
// block index is remapped to give every XCD one contiguous run of blocks,
// taken in dispatch order: the lines two blocks share then meet in one L2
// instead of being fetched from HBM by two. A bijection on [0, nb).
__device__ inline int xcd_block(int b, int nb) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, per = nb / kXcd, extra = nb % kXcd;
  return x * per + min(x, extra) + b / kXcd;
}

// Blocks of the multi-block exclusive scan over m counters (0: one block).
int scan_blocks(int64_t m);

// Small helpers.
hipError_t fill_int(int* ptr, int value, int64_t count, hipStream_t s);
hipError_t fill_double(double* ptr, double value, int64_t count, hipStream_t s);

}  // namespace dpse
