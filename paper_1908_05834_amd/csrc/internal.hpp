// Internal declarations shared by the translation units of libbchar.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bchar.h"

namespace bchar {

// ---------------------------------------------------------------- errors

void set_error(const std::string& msg);

struct Error {
  bchar_status status;
  std::string msg;
};

#define BCHAR_HIP(call)                                                            \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::bchar::Error{BCHAR_E_DEVICE, std::string(#call) + ": " +             \
                                               hipGetErrorString(e_)};             \
  } while (0)

#define BCHAR_REQUIRE(cond, status, msg)                                           \
  do {                                                                             \
    if (!(cond)) throw ::bchar::Error{status, msg};                                \
  } while (0)

// ---------------------------------------------------------------- memory

// Grow-only device buffer.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void reserve(size_t n);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Bump allocator over a list of device chunks, reset at the start of every
// build and kept between builds, so that steady-state builds allocate
// nothing.  Allocations are 256-byte aligned and stay valid until reset.
// `mark()` / `rewind()` free everything allocated after a mark.
struct Arena {
  std::vector<DBuf> chunks;
  size_t cur = 0;   // chunk in use
  size_t off = 0;   // offset in that chunk
  void reset() { cur = 0; off = 0; }
  struct Mark { size_t cur, off; };
  Mark mark() const { return {cur, off}; }
  void rewind(Mark m) { cur = m.cur; off = m.off; }
  template <class T> T* get(size_t n) { return static_cast<T*>(raw(n * sizeof(T))); }
  void* raw(size_t bytes);
  void release();
};

// ---------------------------------------------------------------- handles

}  // namespace bchar

struct bchar_mesh_s {
  int dim = 0;
  int kind = 0;                // BCHAR_MESH_CARTESIAN or BCHAR_MESH_SIMPLEX
  int64_t n[3] = {1, 1, 1};
  double origin[3] = {0, 0, 0};
  double h[3] = {1, 1, 1};
  double box_lo[3] = {0, 0, 0}, box_hi[3] = {0, 0, 0};   // domain box
  int layout = 0;
  int64_t n_cells = 0, n_balls = 0;
  int nbpc = 1;                // balls per cell; 0: varies (ball_ptr)
  double rmax = 0;             // largest ball radius
  double hash_scale = 1.0;     // bucket side of the hash / (2 rmax)
  bool r_uniform = false;      // every ball has radius r0
  double r0 = 0;
  bool phi_const = true;
  double phi0 = 1;
  double bmax = 0;             // max |K|_phi
  // device arrays
  bchar::DBuf phi;             // n_cells
  bchar::DBuf b;               // n_cells, |K|_phi
  bchar::DBuf rho;             // n_cells, porous density rho_K
  bchar::DBuf rad;             // n_balls, radius
  bchar::DBuf bvol;            // n_balls, |B|
  bchar::DBuf cen;             // dim * n_balls, ball order, fp64
  bchar::DBuf cen32;           // dim * n_balls, fp32
  // simplicial meshes: vertices (SoA), cells ((dim+1) ids per cell) and a
  // uniform grid listing the cells whose bounding box meets each grid cell
  int64_t n_vertices = 0;
  bchar::DBuf vtx;             // dim * n_vertices
  bchar::DBuf cell_cen;        // dim * n_cells, centroids (SoA)
  bchar::DBuf cells;           // int32 (dim + 1) * n_cells, cell-major
  double pl_inv = 0;           // 1 / grid side
  int64_t pl_nb[3] = {1, 1, 1};
  bchar::DBuf pl_start;        // int32 [grid cells + 1]
  bchar::DBuf pl_list;         // int32 cell ids, ascending within a grid cell
  // spatial hash of the residing balls
  double hs = 0;               // bucket side
  int64_t nbk[3] = {1, 1, 1};
  int64_t n_buckets = 0;
  bchar::DBuf bucket_start;    // int32 [n_buckets + 1]
  bchar::DBuf bk_cen;          // fp64 dim * n_balls, bucket order
  bchar::DBuf bk_cen32;        // fp32 dim * n_balls, bucket order
  bchar::DBuf bk_ball;         // int32 n_balls: ball id of each bucket slot
  bchar::DBuf bk_rad;          // fp64 n_balls, radius, bucket order
  bchar::DBuf bk_cell;         // int32 n_balls: cell of each bucket slot
  bchar::DBuf bk_w;            // fp64 n_balls: rho_M phi_M of each bucket slot
  // layouts with a varying number of balls per cell: first ball of every
  // cell, cell of every ball, and tiles of whole cells with at most 256
  // balls each (first cell of every tile)
  // ghost cells (Cartesian, n_ghost layers on every side): flag per cell
  // (uint8), empty when there are none
  int64_t n_ghost = 0;
  bchar::DBuf ghost;           // uint8 n_cells
  bchar::DBuf ball_ptr;        // int32 n_cells + 1
  bchar::DBuf ball_cell;       // int32 n_balls
  bchar::DBuf tile_cell;       // int32 n_tiles + 1
  int64_t n_tiles = 0;
  // scratch of the mesh creation and of bchar_mass
  bchar::Arena ws;
  bchar::DBuf scratch_small;   // small device scalars
};

struct bchar_transfer_s {
  bchar_mesh_s* mesh = nullptr;
  int stage = 0;
  int64_t nnz = 0, n_pairs = 0;
  bchar::DBuf row_ptr;   // int32 n_cells + 1
  bchar::DBuf col;       // int32 nnz
  bchar::DBuf V;         // fp64 nnz, A^(0)
  bchar::DBuf AN;        // fp64 nnz, A^(N)
  bchar::DBuf A;         // fp64 nnz, final
  bchar::DBuf x;         // fp64 nnz
  bchar::DBuf mu, nu;    // fp64 n_cells
  bchar::DBuf zdual;     // fp64 4 n_cells: per-cell multipliers (s, g) of the last
                         // solve, leading parts then compensations
  int warm_level = -1;   // box level of the last converged solve
  int warm_newton_skip = 0;  // rebuilds left that start with the warm interior point
                             // (the semismooth warm attempt recently failed before
                             // taking a step)
  bchar::DBuf tracked;   // fp64 dim * n_balls
  bchar::DBuf r_hat;     // fp64 n_balls
  bchar::DBuf lam;       // fp64 n_balls, log growth (non-solenoidal builds)
  bchar::DBuf b_row;     // fp64 n_cells, row targets (non-solenoidal builds)
  bool general = false;  // the last build took a non-solenoidal u
  int64_t groups = 0;    // components of the pattern (non-solenoidal builds)
  bchar::DBuf grp_lab, grp_ptr, grp_perm;   // int32 2n, 2n + 1, 2n (groups > 1)
  bchar::DBuf pair_a, pair_b;  // int32 n_pairs (keep_pairs), any order
  bchar::DBuf stage_col;       // assembly staging: rows in tile order
  bchar::DBuf stage_val;
  int64_t stage_need = 0, pair_need = 0;   // staging room the last builds needed
  int64_t n_void_rows = 0;     // of the last assembly
  bchar_stats stats{};
  // scratch of this transfer's builds (its own, so that builds of several
  // transfers of one mesh may run at once on different streams)
  bchar::Arena ws;
  int substeps = 1;       // sub-steps of dt / substeps after void halvings
  bchar::DBuf cscratch;   // fp64 n_cells, the update's intermediate vector
};

namespace bchar {

// ---------------------------------------------------------------- kernels (host launchers)

// utilities (util.hip)
int64_t exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, Arena& ws,
                           hipStream_t s);          // returns total (syncs)
void exclusive_scan_i32_async(const int32_t* in, int32_t* out, int64_t n, Arena& ws,
                              hipStream_t s);        // total at out[n]
// Stable counting sort of item ids 0..n-1 by key[i] in [0, nkeys):
// ptr[nkeys+1], perm[n] with items of each key in ascending id order.
void bucket_sort(const int32_t* key, int64_t n, int64_t nkeys, int32_t* ptr, int32_t* perm,
                 Arena& ws, hipStream_t s);
double max_abs(const double* v, int64_t n, Arena& ws, hipStream_t s);   // syncs
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void fill_f64(double* p, double v, int64_t n, hipStream_t s);

// mesh (mesh.hip)
// Cartesian layouts: every ball of radius r and measure ball_vol, rho and
// |K| the same on every cell
struct UniformBalls {
  double r, ball_vol, rho, cell_vol;
};
// centres, radii, measures, rho and |K|_phi of a Cartesian layout on the
// device, then the hash
void mesh_build_cartesian(bchar_mesh_s* m, const UniformBalls& u, hipStream_t s);
// the spatial hash of the balls already in cen / rad (side 2 rmax over the
// domain box)
void mesh_build_hash(bchar_mesh_s* m, hipStream_t s);

// tracking + V (build.hip)
struct BuildOut {
  int32_t* row_ptr;    // n_cells + 1 (device)
  int32_t* col;
  double* V;
  int64_t nnz, n_pairs;
  int32_t* pair_a;     // optional
  int32_t* pair_b;
};
// lam: non-null for a non-solenoidal u, receives the log growth of every
// tracked ball (r_hat then always from the cardinal points)
void trace_balls(const bchar_mesh_s* m, const bchar_velocity& u, double dt, int substeps,
                 int precision, double* tracked, double* r_hat, double* lam, Arena& ws,
                 hipStream_t s);
// Row targets of a non-solenoidal step into b_row (after the assembly:
// the components of V's pattern); syncs.
struct TargetInfo {
  double scale = 1.0;   // sum |M|_phi / sum T_K over the whole domain
  int64_t groups = 0;   // connected components of the pattern
  int rounds = 0;       // hook-and-compress rounds that found them
};
// With several components the labels and the grouping are left in
// t->grp_lab, t->grp_ptr, t->grp_perm.
TargetInfo row_targets(const bchar_mesh_s* m, bchar_transfer_s* t, const double* lam,
                       double* b_row, Arena& ws, hipStream_t s);
// Returns BCHAR_OK or VOID_ROW (first_void set); allocates the CSR in t.
// lam: per-ball log growth (non-solenoidal u) or null.
bchar_status assemble_v(bchar_mesh_s* m, const double* tracked, const double* r_hat,
                        const double* lam, int precision, bool keep_pairs, bool lds_stage,
                        int tile_aspect, bchar_transfer_s* t, int64_t* first_void,
                        hipStream_t s);

// scaling (scaling.hip)
struct Csc {
  int32_t* ptr;    // n + 1
  int32_t* row;    // nnz: row of each entry, column-major order
  int32_t* pos;    // nnz: CSR position of each entry
};
void build_csc(const int32_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz, Csc& c,
               Arena& ws, hipStream_t s);
// b_row: row targets (|K|_phi for a solenoidal u); columns take |M|_phi
bchar_status scaling_sweeps(const bchar_mesh_s* m, const int32_t* row_ptr, const int32_t* col,
                            const Csc& csc, const double* V, const double* b_row, int64_t nnz,
                            int n_sweeps, double* AN, int64_t* void_col, int64_t* n_void_cols,
                            double* max_col_err, Arena& ws, hipStream_t s);

// QP (qp.hip)
struct QpResult {
  int level = 0, newton = 0, cg = 0, ipm = 0;
  int64_t coarse_bytes = 0;   // bytes one coarse-level cycle moves at least
  int64_t smooth_bytes = 0;   // bytes a launched-level sweep moves at least, mean
                              // over the sweeps of one cycle
  double residual = 0;
  int64_t at_lower = 0, at_upper = 0;
  bool corrected = false;     // the answer came from the equality correction
};
// zdual: per-cell multipliers (s, g), 2 n leading parts and 2 n
// compensations kept by the transfer;
// warm_level: box level of the previous converged solve, or -1;
// warm_newton_skip: solves left that skip the semismooth warm attempt (set
// to kWarmNewtonPause when it fails before its first step, counted down by
// each warm solve).
// The connected components of the bipartite graph of the pattern (rows
// 0..n-1, columns n..2n-1): every node's label (the smallest node of its
// component) and the nodes grouped by label (ptr: 2n + 1, perm: 2n).
struct Groups {
  const int32_t* lab;
  const int32_t* ptr;
  const int32_t* perm;
};
// groups: the components when there are several (their null directions
// are projected out of every Newton system), else null
bchar_status solve_qp(const bchar_mesh_s* m, const int32_t* row_ptr, const int32_t* col,
                      const Csc& csc, const double* AN, const double* b_row,
                      const Groups* groups, int64_t nnz, const bchar_opts& o, double* x,
                      double* mu, double* nu, double* A, double* zdual, int warm_level,
                      int& warm_newton_skip, QpResult& res, Arena& ws, hipStream_t s);

// apply / mass (apply.hip)
void apply_transfer(const bchar_transfer_s* t, const double* cin, double* cout, hipStream_t s);
double porous_mass(const bchar_mesh_s* m, const double* c, Arena& ws, hipStream_t s);
// the same sum into device memory, asynchronous, allocating nothing (its
// partials use a file-scope device array shared by every call on a GPU)
void porous_mass_into(const bchar_mesh_s* m, const double* c, double* d_out, hipStream_t s);

// ---------------------------------------------------------------- small helpers

inline unsigned blocks_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

}  // namespace bchar

namespace bchar {

// ---------------------------------------------------------------- kernel timing
//
// When enabled for a kernel name, every launch of that kernel (or every
// `every`-th) is bracketed by two HIP events recorded on its stream;
// bchar_profile_read sums the elapsed times.  Off by default: a disabled
// scope costs one atomic load.
// Opt-in progress trace on stderr (environment variable BCHAR_TRACE=1):
// stage wall times of every build and the solver's iteration counts.
bool trace_enabled();
double wall_seconds();

// Work replayed from a HIP graph cannot carry events: while a graph is
// captured no launch is timed (mode off), and one replayed unit in `every`
// (prof_unit_due) is launched eagerly instead, with every launch of the
// timed kernel in it bracketed (mode all).  The mode is per thread.
enum class ProfMode { normal, off, all };
void prof_set_mode(ProfMode m);
bool prof_unit_due();
struct ProfModeGuard {
  explicit ProfModeGuard(ProfMode m) { prof_set_mode(m); }
  ~ProfModeGuard() { prof_set_mode(ProfMode::normal); }
};

struct ProfScope {
  ProfScope(const char* name, hipStream_t s);
  ~ProfScope();
  void* pair;       // this launch's start/end events in the timing state (null: not timed)
  hipStream_t s;
};

}  // namespace bchar
