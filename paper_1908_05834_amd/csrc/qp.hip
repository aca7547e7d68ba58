// The least-change bounded problem of Sec. 3.2 (eq. opti_masscons).
//
// Unknowns: one x_k per stored entry a_k of A^(N).  Minimise x^T x subject
// to the row sums and column sums of a (1 + x) equal to |K|_phi and
// |M|_phi, and lo <= x <= hi (the paper's box is 0 <= 1 + x <= 2, read as
// -1 <= x <= 1; the relaxation levels drop the cap, then the box).
//
// Method: the minimiser is unique; it is reached through the dual.  With
// multipliers mu (rows) and nu (columns), x_k = clip(a_k (mu_i + nu_j)).
// The dual function is convex and C^1 with gradient F = constraint
// residual.  Semismooth Newton on it converges fast from a good start but
// crawls from a poor one: entries pinned to the box give it no curvature,
// cells of a mesh that barely move link to their neighbours only through
// such entries, some of them tiny, and the multipliers that pin them must
// grow to about 1 / a_k.  So a level with a bound first runs a primal-dual
// interior point (Mehrotra predictor-corrector), whose Newton systems keep
// every entry with a positive weight, and semismooth Newton finishes from
// its t; a rebuild first tries semismooth Newton from the previous
// multipliers.  An interior point that stalls just short of the tolerance
// (systems at the edge of what CG solves) is finished by a least-norm
// correction onto the equalities; on the box x >= -1 an interior point
// that gives up from x = 0 is restarted from the minimiser of the
// equalities alone.  Every Newton system is a weighted bipartite graph
// Laplacian L (d_mu; -d_nu) = (-F_row; F_col), solved by preconditioned
// conjugate gradients in per-cell coordinates.  t_k = a_k (mu_i + nu_j) is
// carried per entry and updated by increments, since the multipliers span
// many orders of magnitude.
//
// Preconditioner: one symmetric two-grid cycle on the bipartite graph
// (weighted Jacobi smoothing; each row node joins the column node it is
// most strongly coupled to, which turns the graph into a graph on cells),
// then a V-cycle of aggregation multigrid on the cell graph: pairwise
// matching along strong couplings (w_pq >= beta max(w_p., w_q.)), Galerkin
// coarse operators, l1-Jacobi smoothing, a dense solve on the coarsest
// level.  The aggregation is fixed once per solve from the all-free
// weights a_k^2; each Newton system refreshes the weights of every level
// (entries on the box weigh 0 in semismooth Newton, a_k^2 D_k in the
// interior point).  Weights span many decades on these
// matrices (cells that barely move couple to their neighbours by slivers),
// which is why plain Jacobi-preconditioned CG does not converge here.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "device_util.hpp"
#include "internal.hpp"

namespace bchar {

constexpr int kT = 256;   // threads per block for vector kernels
constexpr int kRedBlocks = 512;
constexpr int kMaxCoarse = 512;    // dense coarsest solve
constexpr int kAmgCap = 2048;      // candidate entries per coarse node (LDS)
constexpr int kIpmMaxIter = 100;   // interior-point iterations per box level
constexpr double kIpmMuTight = 1e-13;  // complementarity of an accepted interior point
constexpr double kIpmWarmShift = 1e-3; // distance from the box of a warm interior point
constexpr int kIpmInfeasIt = 10;       // iterations before the no-progress test
constexpr double kIpmCgLoose = 1.0;    // CG tolerance of the directions, relative to
constexpr double kIpmCgTight = 1e-2;   // min(|rhs|, mu): first try, and retry
constexpr double kIpmMuFloor = 1e-14;  // complementarity at rounding level
constexpr int kCorrectionSteps = 40;  // Newton steps of the equality correction at most
constexpr double kIpmDiverged = 1e3;   // complementarity growth of an empty-looking box
constexpr double kIpmNearFeasible = 1e-8;  // |B x - r| of an interior point that stalls
                                           // there, handed to the polish and then
                                           // to the equality correction
constexpr int kWarmNewton = 3;     // semismooth steps tried from a warm start
constexpr int kWarmNewtonPause = 3;  // warm solves that skip them after they failed
                                     // without a step
constexpr int kPolishNewton = 6;   // semismooth steps after the interior point
constexpr int kFallbackNewton = 40; // semismooth steps on a level every interior point
                                    // gave up on, and the short steps it may take
constexpr int kFallbackPatience = 8;
constexpr int kFallbackNewtonLong = 100;  // the same from zero on x >= -1 once every
constexpr int kFallbackPatienceLong = 40; // interior point there gave up
constexpr int kCrossoverSteps = 2; // fixed-side Newton steps from an interior point
constexpr int kCrossoverRounds = 4; // active-set updates of the sides after the first
constexpr double kCrossoverRatio = 1e-3;  // slack / multiplier of a pinned entry
constexpr int64_t kZsmoothTwoMaxCells = 1 << 20;  // k_zsmooth_two up to this size
constexpr int kPolishCG = 60;      // CG cap of the warm steps, and of those after an
                                   // interior point that met tol

// ====================================================================== reductions

// Final combine of the per-block partials by one block of kFinalThreads:
// thread i takes the partials i, i + kFinalThreads, ... in order, then a
// fixed tree.  The order is fixed, so the result is reproducible.
constexpr int kFinalThreads = 256;
__device__ __forceinline__ double block_final_sum(const double* __restrict__ part, int np,
                                                  double* sh) {
  CSum acc;
  for (int i = threadIdx.x; i < np; i += kFinalThreads) {
    CSum o;
    o.hi = part[2 * i];
    o.lo = part[2 * i + 1];
    acc.add(o);
  }
  return block_csum(acc, sh).value();
}

__global__ void __launch_bounds__(kFinalThreads) k_reduce_final_sum(
    const double* __restrict__ part, int np, double* __restrict__ out) {
  __shared__ double sh[32];
  const double v = block_final_sum(part, np, sh);
  if (threadIdx.x == 0) out[0] = v;
}

__global__ void k_reduce_final_max(const double* __restrict__ part, int np,
                                   double* __restrict__ out) {
  double m = 0;
  for (int i = threadIdx.x; i < np; i += kWave) m = fmax(m, part[i]);
  m = wave_max(m);
  if (threadIdx.x == 0) out[0] = m;
}

// dot(a, b) over n, compensated, deterministic (fixed grid)
__global__ void __launch_bounds__(kT) k_dot_part(const double* __restrict__ a,
                                                 const double* __restrict__ b, int64_t n,
                                                 double* __restrict__ part) {
  __shared__ double sh[32];
  CSum acc;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    acc.add(a[i] * b[i]);
  CSum t = block_csum(acc, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = t.hi;
    part[2 * blockIdx.x + 1] = t.lo;
  }
}

__global__ void __launch_bounds__(kT) k_sum_part(const double* __restrict__ a, int64_t n,
                                                 double* __restrict__ part) {
  __shared__ double sh[32];
  CSum acc;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    acc.add(a[i]);
  CSum t = block_csum(acc, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = t.hi;
    part[2 * blockIdx.x + 1] = t.lo;
  }
}

__global__ void __launch_bounds__(kT) k_maxabs_part(const double* __restrict__ a, int64_t n,
                                                    double* __restrict__ part) {
  __shared__ double sh[16];
  double m = 0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    m = fmax(m, fabs(a[i]));
  m = block_max(m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

struct Reducer {
  double* part;   // 2 * kRedBlocks
  double* out;    // device scalars
  hipStream_t s;
  // device scalar out[slot] = dot(a, b)
  void dot(const double* a, const double* b, int64_t n, int slot) {
    {
      ::bchar::ProfScope ps_("k_dot_part", s);
      k_dot_part<<<kRedBlocks, kT, 0, s>>>(a, b, n, part);
    }
    {
      ::bchar::ProfScope ps_("k_reduce_final_sum", s);
      k_reduce_final_sum<<<1, kFinalThreads, 0, s>>>(part, kRedBlocks, out + slot);
    }
  }
  void sum(const double* a, int64_t n, int slot) {
    {
      ::bchar::ProfScope ps_("k_sum_part", s);
      k_sum_part<<<kRedBlocks, kT, 0, s>>>(a, n, part);
    }
    {
      ::bchar::ProfScope ps_("k_reduce_final_sum", s);
      k_reduce_final_sum<<<1, kFinalThreads, 0, s>>>(part, kRedBlocks, out + slot);
    }
  }
  void maxabs(const double* a, int64_t n, int slot) {
    {
      ::bchar::ProfScope ps_("k_maxabs_part", s);
      k_maxabs_part<<<kRedBlocks, kT, 0, s>>>(a, n, part);
    }
    {
      ::bchar::ProfScope ps_("k_reduce_final_max", s);
      k_reduce_final_max<<<1, 64, 0, s>>>(part, kRedBlocks, out + slot);
    }
  }
  double fetch(int slot) {
    double v = 0;
    BCHAR_HIP(hipMemcpyAsync(&v, out + slot, sizeof(double), hipMemcpyDeviceToHost, s));
    BCHAR_HIP(hipStreamSynchronize(s));
    return v;
  }
};

// ====================================================================== graph levels

struct Level {
  int64_t n = 0, ne = 0;      // nodes, off-diagonal entries
  int32_t* ptr = nullptr;      // n + 1
  int32_t* nbr = nullptr;      // ne
  double* w = nullptr;         // ne, current weights (>= 0)
  double* w0 = nullptr;        // ne, structural weights (all entries free)
  double* diag = nullptr;      // n: sum w + tau
  double* sdinv = nullptr;     // n: smoother step (omega / d)
  double omega = 1.0;
  bool l1 = true;              // smoother diagonal = diag + sum w (l1-Jacobi)
  int32_t* cnt = nullptr;      // fine nodes merged into each node (null on level 0)
  // aggregation towards the next level
  int32_t* agg = nullptr;      // n
  int32_t* mptr = nullptr;     // next.n + 1
  int32_t* mem = nullptr;      // members, grouped by coarse node
  int32_t* cptr = nullptr;     // next.ne + 1: contributions of each coarse entry
  int32_t* cedge = nullptr;    // this level's edge ids
  // vectors
  double *b = nullptr, *x = nullptr, *x2 = nullptr, *r = nullptr;
  // restricted operator R L (row C: the residual of the aggregate C is
  // sum_{p in C} b_p + sum_k ra_val[k] x[ra_col[k]]), with the
  // contributions of every entry (fine edge e: + w_e; -1 - q: - diag_q)
  int64_t nra = 0;
  int32_t *ra_ptr = nullptr, *ra_col = nullptr, *ra_cptr = nullptr, *ra_code = nullptr;
  double* ra_val = nullptr;
  // the cycle's coarse level: `step` levels down, reached through the
  // composed aggregation (cagg, cmptr, cmem; the level's own maps when
  // step = 1).  Aggregation with piecewise-constant prolongation composes
  // exactly: the Galerkin operator two levels down is that of the composed
  // aggregates, so a cycle may pass over a level.
  int step = 1;
  int32_t *cagg = nullptr, *cmptr = nullptr, *cmem = nullptr;
};

// Levels small enough for one workgroup run in a single launch
// (k_fused_cycle): their descriptions live in device memory.
constexpr int kFusedMaxNodes = 8192;
constexpr int kFusedMaxLevels = 48;
constexpr int kFusedLds = 7168;     // doubles of LDS for two iterates of every fused level
constexpr int kFusedLdsTotal = 20464;  // doubles of LDS of the fused cycle (160 KiB with red)
constexpr int kFusedThreads = 1024;   // the fused cycle's workgroup
constexpr int kTouchRound = 16;       // line loads a thread issues before using them
constexpr int kTouchMax = 512;        // ranges of the touch table

struct FusedLevels {
  int count;                          // fused levels, the last is the coarsest
  int dense;                          // coarsest solved with the inverse G
  int pre, post, coarse_sweeps;
  int n[kFusedMaxLevels];
  const int32_t* ptr[kFusedMaxLevels];
  const int32_t* nbr[kFusedMaxLevels];
  const double* w[kFusedMaxLevels];
  const double* diag[kFusedMaxLevels];
  const double* sdinv[kFusedMaxLevels];
  const int32_t* agg[kFusedMaxLevels];
  const int32_t* mptr[kFusedMaxLevels];
  const int32_t* mem[kFusedMaxLevels];
  double* b[kFusedMaxLevels];
  double* x[kFusedMaxLevels];
  double* x2[kFusedMaxLevels];
  const double* G;
  int off[kFusedMaxLevels];           // offset of each level's x in the x store
  int ne[kFusedMaxLevels];            // edges of each fused level
  int total;                          // sum of n over the fused levels
  int lds;                            // x store in LDS (else gx, global)
  double* gx;                         // global x store, 2 total doubles
  // levels whose graph is copied into LDS at the start of the cycle (row
  // pointers and neighbours as 16-bit, weights as binary64), with the byte
  // offsets of those arrays past the x store
  int gl[kFusedMaxLevels];
  int gptr[kFusedMaxLevels], gnbr[kFusedMaxLevels], gw[kFusedMaxLevels];
  // the same bytes in global memory (rewritten whenever the weights
  // change), so that the cycle copies them into LDS in one coalesced pass
  double2* img;
  int img_vec;                        // 16-byte vectors of the image
  // the arrays the cycle reads from global memory, as ranges of at most
  // kFusedThreads 128-byte lines (a multiple of kTouchRound of them, the
  // padding empty): the cycle touches every line once before its
  // dependent phases
  int ntouch;
  const unsigned char* tbase[kTouchMax];
  int tlines[kTouchMax];
};

// ---------------------------------------------------------------------- level kernels

// diag = sum w + mu * cnt (cnt: fine nodes of the bipartite graph merged
// into the node, so that a shift mu I of the finest operator is carried
// to every level exactly); sdinv = omega / (smoother diagonal)
__global__ void k_level_diag(const int32_t* __restrict__ ptr, const double* __restrict__ w,
                             const int32_t* __restrict__ cnt, int64_t n, double mu,
                             double omega, int l1, double* __restrict__ diag,
                             double* __restrict__ sdinv) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double s = 0;
  for (int32_t e = ptr[p]; e < ptr[p + 1]; ++e) s += w[e];
  const double d = s + (cnt ? mu * (double)cnt[p] : 0.0);
  diag[p] = d;
  const double sd = l1 ? d + s : d;
  sdinv[p] = sd > 0 ? omega / sd : 0.0;
}

// fine-node count of each coarse node
__global__ void k_node_count(const int32_t* __restrict__ mptr, const int32_t* __restrict__ mem,
                             const int32_t* __restrict__ fcnt, int64_t nc,
                             int32_t* __restrict__ cnt) {
  const int64_t C = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= nc) return;
  int32_t c = 0;
  for (int32_t m = mptr[C]; m < mptr[C + 1]; ++m) c += fcnt ? fcnt[mem[m]] : 1;
  cnt[C] = c;
}

// Row kernels of the cell levels give each node kNodeLanes lanes, which
// stride its ~10 edges and combine with xor shuffles in a fixed order: the
// gathers x[nbr[e]] of a node then wait on memory side by side instead of
// one after another.
constexpr int kNodeLanes = 4;

// (L x)[p] - diag[p] x[p] summed over the lanes of node p's group
__device__ __forceinline__ double lanes_offdiag(const int32_t* __restrict__ ptr,
                                                const int32_t* __restrict__ nbr,
                                                const double* __restrict__ w,
                                                const double* __restrict__ x, int64_t p,
                                                int sub, bool live) {
  double s = 0.0;
  if (live) {
    // two of the lane's edges a round, their loads issued together
    const int32_t end = ptr[p + 1];
    int32_t e = ptr[p] + sub;
    for (; e + kNodeLanes < end; e += 2 * kNodeLanes) {
      const int32_t q0 = nbr[e], q1 = nbr[e + kNodeLanes];
      const double w0 = w[e], w1 = w[e + kNodeLanes];
      const double x0 = x[q0], x1 = x[q1];
      s += w0 * x0;
      s += w1 * x1;
    }
    if (e < end) s += w[e] * x[nbr[e]];
  }
  s += __shfl_xor(s, 1, kWave);
  s += __shfl_xor(s, 2, kWave);
  return s;
}

// xo = xi + sdinv (b - L xi)
__global__ void __launch_bounds__(kT) k_smooth(const int32_t* __restrict__ ptr,
                                               const int32_t* __restrict__ nbr,
                                               const double* __restrict__ w,
                                               const double* __restrict__ diag,
                                               const double* __restrict__ sdinv,
                                               const double* __restrict__ b,
                                               const double* __restrict__ xi, int64_t n,
                                               double* __restrict__ xo) {
  const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t p = g / kNodeLanes;
  const int sub = (int)(g % kNodeLanes);
  const bool live = p < n;
  const double off = lanes_offdiag(ptr, nbr, w, xi, p, sub, live);
  if (live && sub == 0) xo[p] = xi[p] + sdinv[p] * (b[p] - (diag[p] * xi[p] - off));
}



// Residual and restriction in one pass through the restricted operator:
// bc[C] = sum_{p in C} b_p + sum_k ra_val[k] x[ra_col[k]], kNodeLanes lanes
// per coarse node (fixed order: lane-strided partial sums, then a
// butterfly); also the coarse level's first Jacobi sweep from zero,
// x1 = sdc bc.
__global__ void __launch_bounds__(kT) k_resid_restrict(
    const int32_t* __restrict__ mptr, const int32_t* __restrict__ mem,
    const double* __restrict__ b, const int32_t* __restrict__ ra_ptr,
    const int32_t* __restrict__ ra_col, const double* __restrict__ ra_val,
    const double* __restrict__ x, int64_t nc, const double* __restrict__ sdc,
    double* __restrict__ bc, double* __restrict__ x1) {
  const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t C = g / kNodeLanes;
  const int sub = (int)(g % kNodeLanes);
  double s = 0.0;
  if (C < nc) {
    for (int32_t m = mptr[C] + sub; m < mptr[C + 1]; m += kNodeLanes) s += b[mem[m]];
    const int32_t end = ra_ptr[C + 1];
    int32_t k = ra_ptr[C] + sub;
    for (; k + kNodeLanes < end; k += 2 * kNodeLanes) {
      const int32_t q0 = ra_col[k], q1 = ra_col[k + kNodeLanes];
      const double v0 = ra_val[k], v1 = ra_val[k + kNodeLanes];
      const double x0 = x[q0], x1 = x[q1];
      s += v0 * x0;
      s += v1 * x1;
    }
    if (k < end) s += ra_val[k] * x[ra_col[k]];
  }
  s += __shfl_xor(s, 1, kWave);
  s += __shfl_xor(s, 2, kWave);
  if (C < nc && sub == 0) {
    bc[C] = s;
    x1[C] = sdc[C] * s;
  }
}

// Values of the restricted operator from the level's weights and diagonal.
__global__ void k_ra_values(const int32_t* __restrict__ ra_cptr,
                            const int32_t* __restrict__ ra_code, const double* __restrict__ w,
                            const double* __restrict__ diag, int64_t nra,
                            double* __restrict__ ra_val) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nra) return;
  double v = 0.0;
  for (int32_t c = ra_cptr[r]; c < ra_cptr[r + 1]; ++c) {
    const int32_t code = ra_code[c];
    v += code >= 0 ? w[code] : -diag[-1 - code];
  }
  ra_val[r] = v;
}

// Pattern of the restricted operator, one coarse node per wave: the
// candidates of each member p (p itself for its diagonal, then the far
// ends of its edges), merged by fine node.  Count pass: row length and
// candidate count.  Fill pass: ascending columns, and the candidates'
// codes grouped by entry.
template <bool FILL>
__global__ void __launch_bounds__(64) k_ra_pattern(
    const int32_t* __restrict__ fptr, const int32_t* __restrict__ fnbr,
    const int32_t* __restrict__ mptr, const int32_t* __restrict__ mem, int64_t nc,
    int32_t* __restrict__ row_cnt, int32_t* __restrict__ cand_cnt,
    const int32_t* __restrict__ ra_ptr, const int32_t* __restrict__ cbase,
    int32_t* __restrict__ ra_col, int32_t* __restrict__ ra_cptr, int32_t* __restrict__ ra_code,
    int32_t* __restrict__ overflow) {
  __shared__ int32_t s_key[kAmgCap];
  __shared__ int32_t s_code[kAmgCap];
  __shared__ int32_t s_first[kAmgCap];
  const int64_t C = blockIdx.x;
  const int lane = threadIdx.x;
  int H = 0;
  for (int32_t m = mptr[C]; m < mptr[C + 1]; ++m) {
    const int32_t p = mem[m];
    const int32_t lo = fptr[p] - 1, hi = fptr[p + 1];
    // slot lo is the diagonal of p, the others its edges
    for (int32_t base = lo; base < hi; base += kWave) {
      const int32_t e = base + lane;
      const int keep = e < hi ? 1 : 0;
      const int incl = wave_incl_scan_i(keep);
      const int tot = __shfl(incl, kWave - 1, kWave);
      if (keep && H + incl - 1 < kAmgCap) {
        s_key[H + incl - 1] = e == lo ? p : fnbr[e];
        s_code[H + incl - 1] = e == lo ? -1 - p : e;
      }
      H += tot;
    }
  }
  if (H > kAmgCap) {
    if (lane == 0) atomicMax(overflow, H);
    return;
  }
  __syncthreads();
  for (int e = lane; e < H; e += kWave) {
    const int32_t k = s_key[e];
    int first = 1;
    for (int j = 0; j < e; ++j)
      if (s_key[j] == k) {
        first = 0;
        break;
      }
    s_first[e] = first;
  }
  __syncthreads();
  if (!FILL) {
    int u = 0;
    for (int e = lane; e < H; e += kWave) u += s_first[e];
    u = wave_sum_i(u);
    if (lane == 0) {
      row_cnt[C] = u;
      cand_cnt[C] = H;
    }
    return;
  }
  const int32_t rb = ra_ptr[C];
  const int32_t cb = cbase[C];
  for (int e = lane; e < H; e += kWave) {
    const int32_t k = s_key[e];
    int less = 0, before = 0, rank = 0;
    for (int j = 0; j < H; ++j) {
      const int32_t kj = s_key[j];
      less += kj < k;
      before += (kj == k) && (j < e);
      rank += s_first[j] && kj < k;
    }
    ra_code[cb + less + before] = s_code[e];
    if (s_first[e]) {
      ra_col[rb + rank] = k;
      ra_cptr[rb + rank] = cb + less;
    }
  }
}


// Prolongation and the first post-smoothing sweep in one pass: y = x +
// xc[agg] is formed where it is gathered, xo = y + sdinv (b - L y)
__global__ void __launch_bounds__(kT) k_prolong_smooth(
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ nbr,
    const double* __restrict__ w, const double* __restrict__ diag,
    const double* __restrict__ sdinv, const double* __restrict__ b,
    const double* __restrict__ x, const int32_t* __restrict__ agg,
    const double* __restrict__ xc, int64_t n, double* __restrict__ xo) {
  const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t p = g / kNodeLanes;
  const int sub = (int)(g % kNodeLanes);
  const bool live = p < n;
  double s = 0.0;
  if (live) {
    const int32_t end = ptr[p + 1];
    int32_t e = ptr[p] + sub;
    for (; e + kNodeLanes < end; e += 2 * kNodeLanes) {
      const int32_t q0 = nbr[e], q1 = nbr[e + kNodeLanes];
      const double w0 = w[e], w1 = w[e + kNodeLanes];
      const int32_t c0 = agg[q0], c1 = agg[q1];
      const double y0 = x[q0] + xc[c0], y1 = x[q1] + xc[c1];
      s += w0 * y0;
      s += w1 * y1;
    }
    if (e < end) {
      const int32_t q = nbr[e];
      s += w[e] * (x[q] + xc[agg[q]]);
    }
  }
  s += __shfl_xor(s, 1, kWave);
  s += __shfl_xor(s, 2, kWave);
  if (live && sub == 0) {
    const double y = x[p] + xc[agg[p]];
    xo[p] = y + sdinv[p] * (b[p] - (diag[p] * y - s));
  }
}

// coarse weights: sum of the fine edge weights of each coarse entry
__global__ void k_coarse_values(const int32_t* __restrict__ cptr,
                                const int32_t* __restrict__ cedge,
                                const double* __restrict__ wf, int64_t ne,
                                double* __restrict__ wc) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ne) return;
  double s = 0;
  for (int32_t c = cptr[r]; c < cptr[r + 1]; ++c) s += wf[cedge[c]];
  wc[r] = s;
}

// ---------------------------------------------------------------------- setup kernels

// Row node i of the bipartite graph joins the column (cell) it is most
// strongly coupled to; column node n + j stays with cell j.
__global__ void k_agg_rows(const int32_t* __restrict__ rptr, const int32_t* __restrict__ col,
                           const double* __restrict__ a, int64_t n, int32_t* __restrict__ agg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double best = -1.0;
  int32_t bj = col[rptr[i]];
  for (int32_t k = rptr[i]; k < rptr[i + 1]; ++k) {
    const double v = fabs(a[k]);
    if (v > best) {
      best = v;
      bj = col[k];
    }
  }
  agg[i] = bj;
  agg[n + i] = (int32_t)i;
}

// One coarse node per wave: gather the edges of its members, map their
// far ends to coarse ids, drop internal edges, merge equal coarse
// neighbours.  Count pass: row length and candidate count.  Fill pass:
// sorted neighbours, and the candidate (fine edge) ids grouped by coarse
// entry in ascending order.
template <bool FILL>
__global__ void __launch_bounds__(64) k_galerkin(
    const int32_t* __restrict__ fptr, const int32_t* __restrict__ fnbr,
    const int32_t* __restrict__ agg, const int32_t* __restrict__ mptr,
    const int32_t* __restrict__ mem, int64_t nc, int32_t* __restrict__ row_cnt,
    int32_t* __restrict__ cand_cnt, const int32_t* __restrict__ cptr_row,
    const int32_t* __restrict__ cbase, int32_t* __restrict__ cnbr,
    int32_t* __restrict__ eptr, int32_t* __restrict__ cedge, int32_t* __restrict__ overflow) {
  __shared__ int32_t s_key[kAmgCap];
  __shared__ int32_t s_edge[kAmgCap];
  __shared__ int32_t s_first[kAmgCap];
  const int64_t C = blockIdx.x;
  const int lane = threadIdx.x;
  // candidates of each member, in member order then edge order
  int H = 0;
  for (int32_t m = mptr[C]; m < mptr[C + 1]; ++m) {
    const int32_t p = mem[m];
    const int32_t lo = fptr[p], hi = fptr[p + 1];
    for (int32_t base = lo; base < hi; base += kWave) {
      const int32_t e = base + lane;
      int keep = 0;
      int32_t Q = -1;
      if (e < hi) {
        Q = agg[fnbr[e]];
        keep = Q != (int32_t)C;
      }
      const int incl = wave_incl_scan_i(keep);
      const int tot = __shfl(incl, kWave - 1, kWave);
      if (keep && H + incl - 1 < kAmgCap) {
        s_key[H + incl - 1] = Q;
        s_edge[H + incl - 1] = e;
      }
      H += tot;
    }
  }
  if (H > kAmgCap) {
    if (lane == 0) atomicMax(overflow, H);
    return;
  }
  __syncthreads();
  for (int e = lane; e < H; e += kWave) {
    const int32_t k = s_key[e];
    int first = 1;
    for (int j = 0; j < e; ++j)
      if (s_key[j] == k) {
        first = 0;
        break;
      }
    s_first[e] = first;
  }
  __syncthreads();
  if (!FILL) {
    int u = 0;
    for (int e = lane; e < H; e += kWave) u += s_first[e];
    u = wave_sum_i(u);
    if (lane == 0) {
      row_cnt[C] = u;
      cand_cnt[C] = H;
    }
    return;
  }
  const int32_t rb = cptr_row[C];
  const int32_t cb = cbase[C];
  for (int e = lane; e < H; e += kWave) {
    const int32_t k = s_key[e];
    int less = 0, before = 0, rank = 0;
    for (int j = 0; j < H; ++j) {
      const int32_t kj = s_key[j];
      less += kj < k;
      before += (kj == k) && (j < e);
      rank += s_first[j] && kj < k;
    }
    cedge[cb + less + before] = s_edge[e];
    if (s_first[e]) {
      cnbr[rb + rank] = k;
      eptr[rb + rank] = cb + less;
    }
  }
}

__global__ void k_max_w(const int32_t* __restrict__ ptr, const double* __restrict__ w,
                        int64_t n, double* __restrict__ mx) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double m = 0;
  for (int32_t e = ptr[p]; e < ptr[p + 1]; ++e) m = fmax(m, w[e]);
  mx[p] = m;
}

// matching round: unmatched p proposes to its strongest unmatched,
// symmetrically strong neighbour (ties to the smaller id)
__global__ void k_propose(const int32_t* __restrict__ ptr, const int32_t* __restrict__ nbr,
                          const double* __restrict__ w, const double* __restrict__ mx,
                          const int32_t* __restrict__ partner, double beta, int64_t n,
                          int32_t* __restrict__ prop) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int32_t best = -1;
  double bw = 0;
  if (partner[p] < 0) {
    for (int32_t e = ptr[p]; e < ptr[p + 1]; ++e) {
      const int32_t q = nbr[e];
      if (q == p || partner[q] >= 0) continue;
      const double v = w[e];
      if (!(v > 0) || v < beta * mx[p] || v < beta * mx[q]) continue;
      if (v > bw || (v == bw && q < best)) {
        bw = v;
        best = q;
      }
    }
  }
  prop[p] = best;
}

__global__ void k_accept(const int32_t* __restrict__ prop, int64_t n,
                         int32_t* __restrict__ partner) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t q = prop[p];
  if (q >= 0 && prop[q] == (int32_t)p) partner[p] = q;
}

// An unmatched node joins the aggregate of its strongest matched
// neighbour when that coupling is strong for it (>= beta of its strongest).
__global__ void k_join(const int32_t* __restrict__ ptr, const int32_t* __restrict__ nbr,
                       const double* __restrict__ w, const double* __restrict__ mx,
                       const int32_t* __restrict__ partner, double beta, int64_t n,
                       int32_t* __restrict__ target) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int32_t best = -1;
  if (partner[p] < 0) {
    double bw = 0;
    for (int32_t e = ptr[p]; e < ptr[p + 1]; ++e) {
      const int32_t q = nbr[e];
      if (q == p || partner[q] < 0) continue;
      const double v = w[e];
      if (!(v > 0) || v < beta * mx[p]) continue;
      if (v > bw || (v == bw && q < best)) {
        bw = v;
        best = q;
      }
    }
  }
  target[p] = best;
}

// representative of the aggregate of p: the smaller node of its pair, the
// pair it joined, or itself
__device__ __forceinline__ int32_t agg_rep(const int32_t* partner, const int32_t* target,
                                           int32_t p) {
  int32_t q = partner[p];
  if (q >= 0) return p < q ? p : q;
  const int32_t t = target[p];
  if (t >= 0) {
    q = partner[t];
    return t < q ? t : q;
  }
  return p;
}

__global__ void k_rep_flag(const int32_t* __restrict__ partner,
                           const int32_t* __restrict__ target, int64_t n,
                           int32_t* __restrict__ flag) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  flag[p] = agg_rep(partner, target, (int32_t)p) == (int32_t)p ? 1 : 0;
}

__global__ void k_pair_agg(const int32_t* __restrict__ partner,
                           const int32_t* __restrict__ target, const int32_t* __restrict__ cid,
                           int64_t n, int32_t* __restrict__ agg) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  agg[p] = cid[agg_rep(partner, target, (int32_t)p)];
}

// ---------------------------------------------------------------------- coarsest

// Inverse of the coarsest matrix plus a relative shift, by Gauss-Jordan
// elimination in place (the matrix is symmetric positive definite, so no
// pivoting), one workgroup.
// aggregation two levels down: cagg[p] = agg1[agg0[p]]
__global__ void k_compose_agg(const int32_t* __restrict__ agg0, const int32_t* __restrict__ agg1,
                              int64_t n, int32_t* __restrict__ cagg) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) cagg[p] = agg1[agg0[p]];
}

__global__ void __launch_bounds__(1024) k_coarse_inverse(const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ nbr,
                                                         const double* __restrict__ w,
                                                         const double* __restrict__ diag,
                                                         int n, double* __restrict__ G) {
  __shared__ double f[kMaxCoarse];
  __shared__ double s_piv;
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) G[e] = 0.0;
  __syncthreads();
  if (tid == 0) {
    double m = 0;
    for (int p = 0; p < n; ++p) m = fmax(m, diag[p]);
    s_piv = m > 0 ? m : 1.0;
  }
  __syncthreads();
  const double shift = 1e-12 * s_piv;
  for (int p = tid; p < n; p += nt) {
    G[p * n + p] = diag[p] + shift;
    for (int32_t e = ptr[p]; e < ptr[p + 1]; ++e) G[p * n + nbr[e]] -= w[e];
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid == 0) s_piv = G[k * n + k];
    for (int i = tid; i < n; i += nt) f[i] = G[i * n + k];
    __syncthreads();
    const double piv = s_piv;
    for (int j = tid; j < n; j += nt) G[k * n + j] = (j == k ? 1.0 : G[k * n + j]) / piv;
    __syncthreads();
    for (int e = tid; e < n * n; e += nt) {
      const int i = e / n, j = e % n;
      if (i == k) continue;
      G[e] = (j == k ? 0.0 : G[e]) - f[i] * G[k * n + j];
    }
    __syncthreads();
  }
}

// sum over the fused cycle's workgroup (every thread gets it)
__device__ __forceinline__ double block_sum_fused(double v, double* red) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double r = 0;
  for (int i = 0; i < (int)(blockDim.x / kWave); ++i) r += red[i];
  __syncthreads();
  return r;
}

// (b - L x)[p] for one node (graph indices 32-bit in global memory or
// 16-bit in LDS)
template <class I>
__device__ __forceinline__ double lap_resid(const I* ptr, const I* nbr, const double* w,
                                            const double* diag, const double* b,
                                            const double* x, int p) {
  double s = diag[p] * x[p];
  int e = (int)ptr[p];
  const int end = (int)ptr[p + 1];
  // four edges a round, their loads issued together (same summation order)
  for (; e + 4 <= end; e += 4) {
    const int q0 = (int)nbr[e], q1 = (int)nbr[e + 1], q2 = (int)nbr[e + 2], q3 = (int)nbr[e + 3];
    const double w0 = w[e], w1 = w[e + 1], w2 = w[e + 2], w3 = w[e + 3];
    const double x0 = x[q0], x1 = x[q1], x2 = x[q2], x3 = x[q3];
    s -= w0 * x0;
    s -= w1 * x1;
    s -= w2 * x2;
    s -= w3 * x3;
  }
  for (; e < end; ++e) s -= w[e] * x[nbr[e]];
  return b[p] - s;
}

// The LDS image of the graphs of the levels marked gl (16-bit row pointers
// and neighbours, binary64 weights, at the offsets gptr / gnbr / gw).
__global__ void k_fused_image(const FusedLevels* __restrict__ F) {
  unsigned char* img = reinterpret_cast<unsigned char*>(F->img);
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int ng = gridDim.x * blockDim.x;
  for (int l = 0; l < F->count; ++l) {
    if (!F->gl[l]) continue;
    uint16_t* p16 = reinterpret_cast<uint16_t*>(img + F->gptr[l]);
    uint16_t* n16 = reinterpret_cast<uint16_t*>(img + F->gnbr[l]);
    double* w = reinterpret_cast<double*>(img + F->gw[l]);
    const int32_t *gp = F->ptr[l], *gn = F->nbr[l];
    const double* gw = F->w[l];
    for (int p = g; p <= F->n[l]; p += ng) p16[p] = (uint16_t)gp[p];
    for (int e = g; e < F->ne[l]; e += ng) {
      n16[e] = (uint16_t)gn[e];
      w[e] = gw[e];
    }
  }
}

// The V-cycle below and including the first fused level, in one workgroup.
// On entry F->b[0] holds that level's right-hand side; on exit F->x[0]
// holds the cycle's result.  Two iterates of every fused level live in LDS
// when they fit (F->lds), so that the gathers x[nbr[e]] of the smoothing
// sweeps hit LDS and a Jacobi sweep is one pass and one barrier; the
// graphs and right-hand sides stay in global memory (independent loads).
// Every dependent phase is separated by a workgroup barrier.
__global__ void __launch_bounds__(kFusedThreads) k_fused_cycle(const FusedLevels* __restrict__ F) {
  __shared__ double red[16];
  __shared__ __attribute__((aligned(16))) double sh[kFusedLdsTotal];
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int L = F->count;
  double* xs = F->lds ? sh : F->gx;
  unsigned char* gbase = reinterpret_cast<unsigned char*>(sh + (F->lds ? 2 * F->total : 0));
  // Graphs of the levels marked gl: copied into LDS from their image (one
  // coalesced pass, four 16-byte vectors a round, loads first).  The other
  // levels' arrays are touched once per 128-byte line, so that they are in
  // L2 before the dependent phases below: the kernels of the finer levels
  // have streamed them out since the previous cycle.
  {
    const double2* src = F->img;
    double2* dst = reinterpret_cast<double2*>(gbase);
    const int nv = F->img_vec;
    int i = tid;
    for (; i + 3 * nt < nv; i += 4 * nt) {
      const double2 a0 = src[i], a1 = src[i + nt], a2 = src[i + 2 * nt], a3 = src[i + 3 * nt];
      dst[i] = a0;
      dst[i + nt] = a1;
      dst[i + 2 * nt] = a2;
      dst[i + 3 * nt] = a3;
    }
    for (; i < nv; i += nt) dst[i] = src[i];
    // thread tid reads line tid of every range, kTouchRound ranges' loads
    // issued before any is used
    int acc = 0;
    for (int r = 0; r < F->ntouch; r += kTouchRound) {
      int v[kTouchRound];
#pragma unroll
      for (int u = 0; u < kTouchRound; ++u)
        v[u] = tid < F->tlines[r + u]
                   ? *reinterpret_cast<const int*>(F->tbase[r + u] + (size_t)tid * 128)
                   : 0;
#pragma unroll
      for (int u = 0; u < kTouchRound; ++u) acc += v[u];
    }
    // a store that never happens keeps the loads
    if (acc == -1) red[0] = acc;
  }
  __syncthreads();
  // level l's current iterate is xs + off[l] + (par[l] ? total : 0)
  int par[kFusedMaxLevels];
  for (int l = 0; l < L; ++l) par[l] = 0;
  auto X = [&](int l) { return xs + F->off[l] + (par[l] ? F->total : 0); };
  // (b - L x)[p] of level l, from the graph wherever it lives
  auto resid = [&](int l, const double* x, int p) {
    if (F->gl[l])
      return lap_resid(reinterpret_cast<const uint16_t*>(gbase + F->gptr[l]),
                       reinterpret_cast<const uint16_t*>(gbase + F->gnbr[l]),
                       reinterpret_cast<const double*>(gbase + F->gw[l]), F->diag[l], F->b[l],
                       x, p);
    return lap_resid(F->ptr[l], F->nbr[l], F->w[l], F->diag[l], F->b[l], x, p);
  };
  // one damped Jacobi sweep of level l into its other buffer
  auto sweep = [&](int l) {
    const int n = F->n[l];
    const double* sd = F->sdinv[l];
    const double* x = X(l);
    double* y = xs + F->off[l] + (par[l] ? 0 : F->total);
    for (int p = tid; p < n; p += nt) y[p] = x[p] + sd[p] * resid(l, x, p);
    par[l] ^= 1;
    __syncthreads();
  };
  // downward: pre-smoothing (the first sweep from zero is x = sdinv b) and
  // restriction of the residual.  The residual of every node is formed in
  // parallel into the level's spare buffer, then summed per aggregate (in
  // member order) by the coarse node's thread, which also starts the next
  // level's smoothing.
  {
    const double *sd = F->sdinv[0], *b = F->b[0];
    double* x = X(0);
    for (int p = tid; p < F->n[0]; p += nt) x[p] = sd[p] * b[p];
  }
  __syncthreads();
  for (int l = 0; l + 1 < L; ++l) {
    const int n = F->n[l];
    for (int k = 1; k < F->pre; ++k) sweep(l);
    const double* x = X(l);
    double* r = xs + F->off[l] + (par[l] ? 0 : F->total);
    for (int p = tid; p < n; p += nt) r[p] = resid(l, x, p);
    __syncthreads();
    const int nc = F->n[l + 1];
    const int32_t *mptr = F->mptr[l], *mem = F->mem[l];
    const double* sdc = F->sdinv[l + 1];
    double* bc = F->b[l + 1];
    double* xc = X(l + 1);
    for (int C = tid; C < nc; C += nt) {
      double acc = 0;
      int m = mptr[C];
      const int me = mptr[C + 1];
      for (; m + 4 <= me; m += 4) {
        const int p0 = mem[m], p1 = mem[m + 1], p2 = mem[m + 2], p3 = mem[m + 3];
        acc += r[p0];
        acc += r[p1];
        acc += r[p2];
        acc += r[p3];
      }
      for (; m < me; ++m) acc += r[mem[m]];
      bc[C] = acc;
      xc[C] = sdc[C] * acc;
    }
    __syncthreads();
  }
  // coarsest
  {
    const int l = L - 1;
    const int n = F->n[l];
    const double* b = F->b[l];
    double* x = X(l);
    if (F->dense) {
      // x = G (b - mean b), then its mean removed: G carries the nearly
      // singular constant mode with a huge weight, which the mean-free
      // right-hand side leaves out and the last step discards (folding the
      // projections into G instead cancels catastrophically).  16 lanes per
      // row, rows strided over the groups (the 16 lanes of a group share
      // i, so each shuffle stays in a group whose lanes are all active)
      double sb = 0;
      for (int p = tid; p < n; p += nt) sb += b[p];
      const double bmean = block_sum_fused(sb, red) / n;
      constexpr int kRowLanes = 16;
      const int sub = tid % kRowLanes;
      double sx = 0;
      for (int i = tid / kRowLanes; i < n; i += nt / kRowLanes) {
        double acc = 0;
        for (int j = sub; j < n; j += kRowLanes) acc += F->G[i * n + j] * (b[j] - bmean);
        for (int o = kRowLanes / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
        if (sub == 0) {
          x[i] = acc;
          sx += acc;
        }
      }
      const double xmean = block_sum_fused(sx, red) / n;
      for (int i = tid; i < n; i += nt) x[i] -= xmean;
      __syncthreads();
    } else {
      // x = sdinv b was set with the restriction
      for (int k = 1; k < F->coarse_sweeps; ++k) sweep(l);
    }
  }
  // upward: prolongation and post-smoothing
  for (int l = L - 2; l >= 0; --l) {
    const int n = F->n[l];
    const int32_t* agg = F->agg[l];
    double* x = X(l);
    const double* e = X(l + 1);
    for (int p = tid; p < n; p += nt) x[p] += e[agg[p]];
    __syncthreads();
    for (int k = 0; k < F->post; ++k) sweep(l);
  }
  {
    const double* x = X(0);
    for (int p = tid; p < F->n[0]; p += nt) F->x[0][p] = x[p];
  }
}

// ====================================================================== hierarchy

struct Hierarchy {
  std::vector<Level> lv;
  double mu = 0.0;       // shift mu I of the bipartite operator (all levels)
  double* G = nullptr;   // inverse of the shifted coarsest matrix
  int coarse_n = 0;
  bool dense = false;
  int pre = 1, post = 1;             // sweeps of the fused coarse levels
  int coarse_sweeps = 40;
  size_t fused_first = 0;          // first level handled by k_fused_cycle
  int skip = 0;                    // launched levels from this one pass over every other
                                   // level (0: every level is visited)
  FusedLevels* fused = nullptr;    // device copy
  bool fused_img = false;          // it has an LDS image to refresh
  int64_t fused_bytes = 0;         // bytes one fused cycle reads or writes at least
  int64_t smooth_bytes = 0;        // bytes of a launched-level sweep, mean per launch once
};

static void level_refresh_diag(Level& L, double mu, hipStream_t s) {
  {
    ::bchar::ProfScope ps_("k_level_diag", s);
    k_level_diag<<<blocks_for(L.n, kT), kT, 0, s>>>(L.ptr, L.w, L.cnt, L.n, mu, L.omega, L.l1 ? 1 : 0,
                                                    L.diag, L.sdinv);
  }
  BCHAR_HIP(hipGetLastError());
}

// Build the Galerkin pattern of the next level from `L` and its
// aggregation (agg, mptr, mem); returns the coarse level (pattern only).
static Level galerkin_pattern(Level& L, int64_t nc, Arena& ws, hipStream_t s) {
  Level Cl;
  Cl.n = nc;
  int32_t* row_cnt = ws.get<int32_t>(nc + 1);
  int32_t* cand_cnt = ws.get<int32_t>(nc + 1);
  int32_t* overflow = ws.get<int32_t>(1);
  fill_i32(overflow, 0, 1, s);
  {
    ::bchar::ProfScope ps_("k_galerkin", s);
    k_galerkin<false><<<(unsigned)nc, 64, 0, s>>>(L.ptr, L.nbr, L.agg, L.mptr, L.mem, nc,
                                                  row_cnt, cand_cnt, nullptr, nullptr, nullptr,
                                                  nullptr, nullptr, overflow);
  }
  BCHAR_HIP(hipGetLastError());
  int32_t hov = 0;
  BCHAR_HIP(hipMemcpyAsync(&hov, overflow, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  BCHAR_HIP(hipStreamSynchronize(s));
  if (hov > 0)
    throw Error{BCHAR_E_UNSUPPORTED,
                "aggregation: a coarse node has " + std::to_string(hov) + " candidate entries"};
  Cl.ptr = ws.get<int32_t>(nc + 1);
  int32_t* cbase = ws.get<int32_t>(nc + 1);
  Cl.ne = exclusive_scan_i32(row_cnt, Cl.ptr, nc, ws, s);
  const int64_t ncand = exclusive_scan_i32(cand_cnt, cbase, nc, ws, s);
  Cl.nbr = ws.get<int32_t>(Cl.ne + 1);
  L.cptr = ws.get<int32_t>(Cl.ne + 1);
  L.cedge = ws.get<int32_t>(ncand + 1);
  {
    ::bchar::ProfScope ps_("k_galerkin", s);
    k_galerkin<true><<<(unsigned)nc, 64, 0, s>>>(L.ptr, L.nbr, L.agg, L.mptr, L.mem, nc, nullptr,
                                                 nullptr, Cl.ptr, cbase, Cl.nbr, L.cptr, L.cedge,
                                                 overflow);
  }
  BCHAR_HIP(hipGetLastError());
  // closing entry of the contribution pointer
  BCHAR_HIP(hipMemcpyAsync(L.cptr + Cl.ne, cbase + nc, sizeof(int32_t), hipMemcpyDeviceToDevice,
                           s));
  Cl.w = ws.get<double>(Cl.ne + 1);
  Cl.w0 = ws.get<double>(Cl.ne + 1);
  {
    ::bchar::ProfScope ps_("k_coarse_values", s);
    k_coarse_values<<<blocks_for(Cl.ne, kT), kT, 0, s>>>(L.cptr, L.cedge, L.w0, Cl.ne, Cl.w0);
  }
  Cl.cnt = ws.get<int32_t>(nc + 1);
  {
    ::bchar::ProfScope ps_("k_node_count", s);
    k_node_count<<<blocks_for(nc, kT), kT, 0, s>>>(L.mptr, L.mem, L.cnt, nc, Cl.cnt);
  }
  BCHAR_HIP(hipGetLastError());
  return Cl;
}

// Pattern of the restricted operator of level L (aggregates of L, nc of
// them) and the codes its values are summed from.
static void ra_pattern(Level& L, int64_t nc, Arena& ws, hipStream_t s) {
  int32_t* row_cnt = ws.get<int32_t>(nc + 1);
  int32_t* cand_cnt = ws.get<int32_t>(nc + 1);
  int32_t* overflow = ws.get<int32_t>(1);
  fill_i32(overflow, 0, 1, s);
  {
    ::bchar::ProfScope ps_("k_ra_pattern", s);
    k_ra_pattern<false><<<(unsigned)nc, 64, 0, s>>>(L.ptr, L.nbr, L.cmptr, L.cmem, nc, row_cnt,
                                                    cand_cnt, nullptr, nullptr, nullptr,
                                                    nullptr, nullptr, overflow);
  }
  BCHAR_HIP(hipGetLastError());
  int32_t hov = 0;
  BCHAR_HIP(hipMemcpyAsync(&hov, overflow, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  BCHAR_HIP(hipStreamSynchronize(s));
  if (hov > 0)
    throw Error{BCHAR_E_UNSUPPORTED,
                "restriction: an aggregate has " + std::to_string(hov) + " candidate entries"};
  L.ra_ptr = ws.get<int32_t>(nc + 1);
  int32_t* cbase = ws.get<int32_t>(nc + 1);
  L.nra = exclusive_scan_i32(row_cnt, L.ra_ptr, nc, ws, s);
  const int64_t ncand = exclusive_scan_i32(cand_cnt, cbase, nc, ws, s);
  L.ra_col = ws.get<int32_t>(L.nra + 1);
  L.ra_cptr = ws.get<int32_t>(L.nra + 1);
  L.ra_code = ws.get<int32_t>(ncand + 1);
  L.ra_val = ws.get<double>(L.nra + 1);
  {
    ::bchar::ProfScope ps_("k_ra_pattern", s);
    k_ra_pattern<true><<<(unsigned)nc, 64, 0, s>>>(L.ptr, L.nbr, L.cmptr, L.cmem, nc, nullptr,
                                                   nullptr, L.ra_ptr, cbase, L.ra_col, L.ra_cptr,
                                                   L.ra_code, overflow);
  }
  BCHAR_HIP(hipGetLastError());
  // closing entry of the contribution pointer
  BCHAR_HIP(hipMemcpyAsync(L.ra_cptr + L.nra, cbase + nc, sizeof(int32_t),
                           hipMemcpyDeviceToDevice, s));
}

static void alloc_level_vectors(Level& L, Arena& ws) {
  L.diag = ws.get<double>(L.n + 1);
  L.sdinv = ws.get<double>(L.n + 1);
  L.b = ws.get<double>(L.n + 1);
  L.x = ws.get<double>(L.n + 1);
  L.x2 = ws.get<double>(L.n + 1);
  L.r = ws.get<double>(L.n + 1);
}

// Fine level: bipartite graph on 2n nodes (rows, then columns).
static void build_hierarchy(Hierarchy& H, Level fine, const int32_t* rptr, const int32_t* col,
                            const double* a, int64_t n, Arena& ws, hipStream_t s) {
  H.lv.clear();
  fine.omega = 0.6;
  fine.l1 = false;
  alloc_level_vectors(fine, ws);
  H.lv.push_back(fine);
  {
    Level& L = H.lv.back();
    L.agg = ws.get<int32_t>(L.n + 1);
    {
      ::bchar::ProfScope ps_("k_agg_rows", s);
      k_agg_rows<<<blocks_for(n, kT), kT, 0, s>>>(rptr, col, a, n, L.agg);
    }
    BCHAR_HIP(hipGetLastError());
    L.mptr = ws.get<int32_t>(n + 1);
    L.mem = ws.get<int32_t>(L.n + 1);
    bucket_sort(L.agg, L.n, n, L.mptr, L.mem, ws, s);
    Level C = galerkin_pattern(L, n, ws, s);
    C.omega = 1.0;
    C.l1 = true;
    alloc_level_vectors(C, ws);
    H.lv.push_back(C);
  }
  double beta = 0.25;
  while (H.lv.back().n > 128) {
    Level& L = H.lv.back();
    const int64_t nl = L.n;
    double* mx = ws.get<double>(nl + 1);
    int32_t* partner = ws.get<int32_t>(nl + 1);
    int32_t* prop = ws.get<int32_t>(nl + 1);
    {
      ::bchar::ProfScope ps_("k_max_w", s);
      k_max_w<<<blocks_for(nl, kT), kT, 0, s>>>(L.ptr, L.w0, nl, mx);
    }
    fill_i32(partner, -1, nl, s);
    for (int round = 0; round < 10; ++round) {
      {
        ::bchar::ProfScope ps_("k_propose", s);
        k_propose<<<blocks_for(nl, kT), kT, 0, s>>>(L.ptr, L.nbr, L.w0, mx, partner, beta, nl,
                                                    prop);
      }
      {
        ::bchar::ProfScope ps_("k_accept", s);
        k_accept<<<blocks_for(nl, kT), kT, 0, s>>>(prop, nl, partner);
      }
    }
    BCHAR_HIP(hipGetLastError());
    int32_t* target = ws.get<int32_t>(nl + 1);
    {
      ::bchar::ProfScope ps_("k_join", s);
      k_join<<<blocks_for(nl, kT), kT, 0, s>>>(L.ptr, L.nbr, L.w0, mx, partner, beta, nl, target);
    }
    int32_t* flag = ws.get<int32_t>(nl + 1);
    int32_t* cid = ws.get<int32_t>(nl + 1);
    {
      ::bchar::ProfScope ps_("k_rep_flag", s);
      k_rep_flag<<<blocks_for(nl, kT), kT, 0, s>>>(partner, target, nl, flag);
    }
    const int64_t nc = exclusive_scan_i32(flag, cid, nl, ws, s);
    if ((double)nc > 0.97 * (double)nl) break;   // nothing left to aggregate
    if ((double)nc > 0.75 * (double)nl) beta = 0.0;
    L.agg = ws.get<int32_t>(nl + 1);
    {
      ::bchar::ProfScope ps_("k_pair_agg", s);
      k_pair_agg<<<blocks_for(nl, kT), kT, 0, s>>>(partner, target, cid, nl, L.agg);
    }
    L.mptr = ws.get<int32_t>(nc + 1);
    L.mem = ws.get<int32_t>(nl + 1);
    bucket_sort(L.agg, nl, nc, L.mptr, L.mem, ws, s);
    BCHAR_HIP(hipGetLastError());
    Level C = galerkin_pattern(L, nc, ws, s);
    C.omega = 1.0;
    C.l1 = true;
    alloc_level_vectors(C, ws);
    H.lv.push_back(C);
  }
  Level& last = H.lv.back();
  H.coarse_n = (int)last.n;
  H.dense = last.n <= kMaxCoarse;
  if (H.dense) H.G = ws.get<double>((size_t)last.n * last.n + 1);
  // the coarsest cell levels run in one workgroup: as many as keep their
  // iterates (plus a scratch of the largest) within kFusedLds doubles of
  // LDS; if even the coarsest does not fit, the levels of at most
  // kFusedMaxNodes nodes with a global store
  size_t first = H.lv.size() - 1;
  int64_t total = H.lv[first].n;
  const bool lds = 2 * total <= kFusedLds;
  while (first > 1 && H.lv.size() - (first - 1) <= (size_t)kFusedMaxLevels) {
    const int64_t nn = H.lv[first - 1].n;
    if (lds ? 2 * (total + nn) > kFusedLds : nn > kFusedMaxNodes) break;
    total += nn;
    --first;
  }
  H.fused_first = first;
  // the launched levels of the cycle: from level 1, every level, or with
  // skip every other level (aggregates of about four nodes) while that
  // lands at or above the fused levels; each restricts its residual
  // through R L
  int64_t launched = 0;
  H.smooth_bytes = 0;
  for (size_t l = 1; l < first;) {
    Level& L = H.lv[l];
    L.step = (H.skip > 0 && (int)l >= H.skip && l + 2 <= first) ? 2 : 1;
    if (L.step == 2) {
      L.cagg = ws.get<int32_t>(L.n + 1);
      {
        ::bchar::ProfScope ps_("k_compose_agg", s);
        k_compose_agg<<<blocks_for(L.n, kT), kT, 0, s>>>(L.agg, H.lv[l + 1].agg, L.n, L.cagg);
      }
      BCHAR_HIP(hipGetLastError());
      const int64_t nc2 = H.lv[l + 2].n;
      L.cmptr = ws.get<int32_t>(nc2 + 1);
      L.cmem = ws.get<int32_t>(L.n + 1);
      bucket_sort(L.cagg, L.n, nc2, L.cmptr, L.cmem, ws, s);
    } else {
      L.cagg = L.agg;
      L.cmptr = L.mptr;
      L.cmem = L.mem;
    }
    ra_pattern(L, H.lv[l + L.step].n, ws, s);
    // one sweep (k_smooth) of level l reads the row pointers, neighbours
    // and weights, the diagonal, smoother step, right-hand side and
    // iterate, and writes the new iterate: 44 n + 12 ne bytes; two sweeps
    // a level a cycle
    H.smooth_bytes += 44 * L.n + 12 * L.ne;
    ++launched;
    l += L.step;
  }
  if (launched > 0) H.smooth_bytes /= launched;
  FusedLevels hf{};
  hf.count = (int)(H.lv.size() - first);
  hf.dense = H.dense ? 1 : 0;
  hf.pre = H.pre;
  hf.post = H.post;
  hf.coarse_sweeps = H.coarse_sweeps;
  hf.G = H.G;
  hf.total = (int)total;
  hf.lds = lds ? 1 : 0;
  hf.gx = lds ? nullptr : ws.get<double>((size_t)(2 * total));
  // graphs in LDS, from the coarsest level up, while they fit past the
  // iterates (16-bit indices need fewer than 65536 nodes and edges a level)
  int64_t img_bytes = 0;
  {
    // a multiple of 16 bytes, so that the image rounded up to whole
    // 16-byte vectors still fits
    const int64_t avail = lds ? (8 * (int64_t)(kFusedLdsTotal - 2 * total)) / 16 * 16 : 0;
    int64_t used = 0;
    for (int k = (int)(H.lv.size() - first) - 1; k >= 0; --k) {
      const Level& Lk = H.lv[first + k];
      const int64_t pb = ((2 * (Lk.n + 1) + 7) / 8) * 8;
      const int64_t nbb = ((2 * Lk.ne + 7) / 8) * 8;
      const int64_t need = pb + nbb + 8 * Lk.ne;
      const bool fits = lds && Lk.n < 65535 && Lk.ne < 65535 && used + need <= avail;
      hf.gl[k] = fits ? 1 : 0;
      if (!fits) {
        for (int j = k - 1; j >= 0; --j) hf.gl[j] = 0;
        break;
      }
      hf.gptr[k] = (int)used;
      hf.gnbr[k] = (int)(used + pb);
      hf.gw[k] = (int)(used + pb + nbb);
      used += need;
    }
    img_bytes = used;
  }
  hf.img_vec = (int)((img_bytes + 15) / 16);
  hf.img = hf.img_vec > 0 ? ws.get<double2>((size_t)hf.img_vec) : nullptr;
  for (int k = 0, o = 0; k < hf.count; ++k) {
    Level& Lk = H.lv[first + k];
    hf.off[k] = o;
    o += (int)Lk.n;
    hf.ne[k] = (int)Lk.ne;
    hf.n[k] = (int)Lk.n;
    hf.ptr[k] = Lk.ptr;
    hf.nbr[k] = Lk.nbr;
    hf.w[k] = Lk.w;
    hf.diag[k] = Lk.diag;
    hf.sdinv[k] = Lk.sdinv;
    hf.agg[k] = Lk.agg;
    hf.mptr[k] = Lk.mptr;
    hf.mem[k] = Lk.mem;
    hf.b[k] = Lk.b;
    hf.x[k] = Lk.x;
    hf.x2[k] = Lk.x2;
  }
  // bytes one fused cycle must move: each level's graph (index and weight
  // per edge, row pointers), diagonal, smoother step, right-hand side and
  // aggregation, the coarsest inverse, and the result
  H.fused_bytes = 8 * H.lv[first].n;
  for (int k = 0; k < hf.count; ++k) {
    const int64_t nk = hf.n[k], ek = hf.ne[k];
    H.fused_bytes += 12 * ek + 4 * (nk + 1) + 24 * nk;
    if (k + 1 < hf.count) H.fused_bytes += 8 * nk + 4 * (hf.n[k + 1] + 1);
  }
  if (H.dense) H.fused_bytes += 8 * (int64_t)H.coarse_n * H.coarse_n;
  {
    hf.ntouch = 0;
    auto touch = [&](const void* a, int64_t bytes) {
      const unsigned char* base = static_cast<const unsigned char*>(a);
      for (int64_t lines = (bytes + 127) / 128; lines > 0;) {
        const int take = (int)std::min<int64_t>(lines, kFusedThreads);
        if (hf.ntouch >= kTouchMax) throw Error{BCHAR_E_UNSUPPORTED, "fused cycle: touch table"};
        hf.tbase[hf.ntouch] = base;
        hf.tlines[hf.ntouch] = take;
        ++hf.ntouch;
        base += (int64_t)take * 128;
        lines -= take;
      }
    };
    for (int k = 0; k < hf.count; ++k) {
      const int64_t nk = hf.n[k], ek = hf.ne[k];
      touch(hf.diag[k], 8 * nk);
      touch(hf.sdinv[k], 8 * nk);
      if (k + 1 < hf.count) {
        touch(hf.agg[k], 4 * nk);
        touch(hf.mem[k], 4 * nk);
        touch(hf.mptr[k], 4 * (hf.n[k + 1] + 1));
      }
      if (!hf.gl[k]) {
        touch(hf.w[k], 8 * ek);
        touch(hf.nbr[k], 4 * ek);
        touch(hf.ptr[k], 4 * (nk + 1));
      }
    }
    if (H.dense) touch(H.G, 8 * (int64_t)H.coarse_n * H.coarse_n);
    while (hf.ntouch % kTouchRound) {
      if (hf.ntouch >= kTouchMax) throw Error{BCHAR_E_UNSUPPORTED, "fused cycle: touch table"};
      hf.tbase[hf.ntouch] = nullptr;
      hf.tlines[hf.ntouch] = 0;
      ++hf.ntouch;
    }
  }
  H.fused = ws.get<FusedLevels>(1);
  H.fused_img = hf.img_vec > 0;
  BCHAR_HIP(hipMemcpyAsync(H.fused, &hf, sizeof(hf), hipMemcpyHostToDevice, s));
  BCHAR_HIP(hipStreamSynchronize(s));
}

// New weights on every level (fine weights already in lv[0].w).
static void refresh_hierarchy(Hierarchy& H, hipStream_t s) {
  for (size_t l = 0; l < H.lv.size(); ++l) {
    Level& L = H.lv[l];
    if (l > 0) {
      Level& F = H.lv[l - 1];
      {
        ::bchar::ProfScope ps_("k_coarse_values", s);
        k_coarse_values<<<blocks_for(L.ne, kT), kT, 0, s>>>(F.cptr, F.cedge, F.w, L.ne, L.w);
      }
      BCHAR_HIP(hipGetLastError());
    }
    level_refresh_diag(L, H.mu, s);
    if (L.ra_val) {
      {
        ::bchar::ProfScope ps_("k_ra_values", s);
        k_ra_values<<<blocks_for(L.nra, kT), kT, 0, s>>>(L.ra_cptr, L.ra_code, L.w, L.diag,
                                                         L.nra, L.ra_val);
      }
      BCHAR_HIP(hipGetLastError());
    }
  }
  if (H.dense) {
    Level& L = H.lv.back();
    {
      ::bchar::ProfScope ps_("k_coarse_inverse", s);
      k_coarse_inverse<<<1, 1024, 0, s>>>(L.ptr, L.nbr, L.w, L.diag, (int)L.n, H.G);
    }
    BCHAR_HIP(hipGetLastError());
  }
  if (H.fused_img) {
    {
      ::bchar::ProfScope ps_("k_fused_image", s);
      k_fused_image<<<64, kT, 0, s>>>(H.fused);
    }
    BCHAR_HIP(hipGetLastError());
  }
}

// x_l = cycle(b_l); on return H.lv[l].x holds the result.
static void vcycle(Hierarchy& H, size_t l, hipStream_t s) {
  Level& L = H.lv[l];
  if (l >= H.fused_first) {
    // this level and all coarser ones: one workgroup, one launch
    {
      ::bchar::ProfScope ps_("k_fused_cycle", s);
      k_fused_cycle<<<1, kFusedThreads, 0, s>>>(H.fused);
    }
    BCHAR_HIP(hipGetLastError());
    return;
  }
  // two damped Jacobi sweeps before and after the coarse correction, in
  // four launches: both pre-sweeps, residual and restriction, prolongation
  // with the first post-sweep, the second post-sweep (result in L.x)
  Level& C = H.lv[l + L.step];
  const unsigned gl = blocks_for(L.n * kNodeLanes, kT);
  {
    // the first sweep (x1 = sdinv b, in L.x2) came with the restriction
    ::bchar::ProfScope ps_("k_smooth", s);
    k_smooth<<<gl, kT, 0, s>>>(L.ptr, L.nbr, L.w, L.diag, L.sdinv, L.b, L.x2, L.n, L.x);
  }
  {
    ::bchar::ProfScope ps_("k_resid_restrict", s);
    k_resid_restrict<<<blocks_for(C.n * kNodeLanes, kT), kT, 0, s>>>(
        L.cmptr, L.cmem, L.b, L.ra_ptr, L.ra_col, L.ra_val, L.x, C.n, C.sdinv, C.b, C.x2);
  }
  vcycle(H, l + L.step, s);
  {
    ::bchar::ProfScope ps_("k_prolong_smooth", s);
    k_prolong_smooth<<<gl, kT, 0, s>>>(L.ptr, L.nbr, L.w, L.diag, L.sdinv, L.b, L.x, L.cagg, C.x,
                                        L.n, L.x2);
  }
  {
    ::bchar::ProfScope ps_("k_smooth", s);
    k_smooth<<<gl, kT, 0, s>>>(L.ptr, L.nbr, L.w, L.diag, L.sdinv, L.b, L.x2, L.n, L.x);
  }
  BCHAR_HIP(hipGetLastError());
}

// z = M r: one cycle from the fine level
// ====================================================================== per-cell (s, g) space
//
// The Newton system in the multipliers y = (mu, -nu) is the Laplacian of
// the bipartite graph rows-columns.  Rows and columns are both indexed by
// cells; in the coordinates s_K = (y_rK + y_cK)/2, g_K = y_rK - y_cK an
// entry (K, M) of weight w contributes w v v^T with
//     v = e_sK - e_sM + (e_gK + e_gM)/2   (K != M),     v = e_gK   (K == M).
// Cells that barely move carry a weight near 1 on (K, K) and slivers
// elsewhere: in y coordinates their gauge mode (s_K) is lost to rounding;
// here the s part only ever sees the off-diagonal weights.  Every product
// with this matrix is formed entry by entry from (s, g).

struct ZCells {
  int64_t n;
  const int32_t *rptr, *col, *cptr, *crow, *cpos;
  const int32_t* dpos;   // position of (K, K) in row K, or -1
  const int32_t* best;   // strongest column of row K (level-1 aggregate of the row)
  const double* w;       // weights, CSR order (nnz)
  const double* wc;      // weights, CSC order (nnz)
  double* tau_s;         // relative shifts
  double* tau_g;
  double* bi;            // 3 per cell: inverse of the 2x2 cell block (ss, sg, gg)
  const uint8_t* ghost;  // per cell: unconstrained row and column (ghost cell), or null
};

__global__ void k_diag_pos(const int32_t* __restrict__ rptr, const int32_t* __restrict__ col,
                           int64_t n, int32_t* __restrict__ dpos) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t d = -1;
  for (int32_t k = rptr[i]; k < rptr[i + 1]; ++k)
    if (col[k] == (int32_t)i) d = k;
  dpos[i] = d;
}

// per-cell block [[A, B], [B, C]] of J_z (+ shifts) and its inverse
__global__ void k_zcells(ZCells Z, double rel, double mu) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= Z.n) return;
  double R = 0, Cs = 0;
  for (int32_t k = Z.rptr[K]; k < Z.rptr[K + 1]; ++k)
    if (Z.col[k] != (int32_t)K) R += Z.w[k];
  for (int32_t e = Z.cptr[K]; e < Z.cptr[K + 1]; ++e)
    if (Z.crow[e] != (int32_t)K) Cs += Z.wc[e];
  const double wkk = Z.dpos[K] >= 0 ? Z.w[Z.dpos[K]] : 0.0;
  const double A0 = R + Cs;
  const double C0 = wkk + 0.25 * (R + Cs);
  // a relative shift for the exactly singular directions, plus mu I of
  // the (mu, -nu) operator, which reads 2 mu on s and mu / 2 on g
  const double ts = rel * (A0 > 0 ? A0 : 1.0) + 2.0 * mu;
  const double tg = rel * (C0 > 0 ? C0 : 1.0) + 0.5 * mu;
  Z.tau_s[K] = ts;
  Z.tau_g[K] = tg;
  const double A = A0 + ts, C = C0 + tg, B = 0.5 * (R - Cs);
  // A C - B^2 written as a sum of non-negative terms
  const double det = (R + Cs) * wkk + R * Cs + ts * C0 + tg * A0 + ts * tg;
  // a ghost cell's (s, g) stay 0: a zero block keeps every sweep off them
  const bool gh = Z.ghost && Z.ghost[K];
  Z.bi[3 * K + 0] = gh ? 0.0 : C / det;
  Z.bi[3 * K + 1] = gh ? 0.0 : -B / det;
  Z.bi[3 * K + 2] = gh ? 0.0 : A / det;
}

// out = J_z z for cell K
// (J_z v) at cell K, the (s, g) values of v at a cell M given by val(M, s, g)
template <class V>
__device__ __forceinline__ void zapply_cell_v(const ZCells& Z, V val, int64_t K, double& os,
                                              double& og) {
  double sK, gK;
  val((int32_t)K, sK, gK);
  double fr = 0, fc = 0, fd = 0;
  // two entries a round with their loads issued together (same order of
  // accumulation as one at a time)
  constexpr int U = 4;
  const int32_t kend = Z.rptr[K + 1];
  int32_t k = Z.rptr[K];
  for (; k + U - 1 < kend; k += U) {
    int32_t M[U];
    double wv[U], sv[U], gv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      M[u] = Z.col[k + u];
      wv[u] = Z.w[k + u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) val(M[u], sv[u], gv[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (M[u] == (int32_t)K)
        fd = wv[u] * gK;
      else
        fr += wv[u] * ((sK - sv[u]) + 0.5 * (gK + gv[u]));
    }
  }
  for (; k < kend; ++k) {
    const int32_t M = Z.col[k];
    if (M == (int32_t)K) {
      fd = Z.w[k] * gK;
    } else {
      double sM, gM;
      val(M, sM, gM);
      fr += Z.w[k] * ((sK - sM) + 0.5 * (gK + gM));
    }
  }
  const int32_t eend = Z.cptr[K + 1];
  int32_t e = Z.cptr[K];
  for (; e + U - 1 < eend; e += U) {
    int32_t I[U];
    double wv[U], sv[U], gv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      I[u] = Z.crow[e + u];
      wv[u] = Z.wc[e + u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) val(I[u], sv[u], gv[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (I[u] != (int32_t)K) fc += wv[u] * ((sv[u] - sK) + 0.5 * (gv[u] + gK));
  }
  for (; e < eend; ++e) {
    const int32_t I = Z.crow[e];
    if (I != (int32_t)K) {
      double sI, gI;
      val(I, sI, gI);
      fc += Z.wc[e] * ((sI - sK) + 0.5 * (gI + gK));
    }
  }
  os = fr - fc + Z.tau_s[K] * sK;
  og = 0.5 * (fr + fc) + fd + Z.tau_g[K] * gK;
}

__device__ __forceinline__ void zapply_cell(const ZCells& Z, const double* __restrict__ zs,
                                            const double* __restrict__ zg, int64_t K,
                                            double& os, double& og) {
  zapply_cell_v(
      Z,
      [&](int32_t M, double& sv, double& gv) {
        sv = zs[M];
        gv = zg[M];
      },
      K, os, og);
}

// the first block-Jacobi sweep from zero at cell M: x1 = omega B^-1 b
__device__ __forceinline__ void zfirst_sweep(const ZCells& Z, double omega,
                                             const double* __restrict__ b, int32_t M, double& s,
                                             double& g) {
  const double bs = b[M], bg = b[Z.n + M];
  s = omega * (Z.bi[3 * M] * bs + Z.bi[3 * M + 1] * bg);
  g = omega * (Z.bi[3 * M + 1] * bs + Z.bi[3 * M + 2] * bg);
}

// out = J_z z; with `part`, also the compensated block sums of z . out
// (one (hi, lo) pair per block, in block order)
__global__ void __launch_bounds__(kT) k_zop(ZCells Z, const double* __restrict__ z,
                                            double* __restrict__ out, double* __restrict__ part) {
  __shared__ double sh[32];
  const int64_t K = (int64_t)blockIdx.x * kT + threadIdx.x;
  CSum acc;
  if (K < Z.n) {
    double os, og;
    zapply_cell(Z, z, z + Z.n, K, os, og);
    if (Z.ghost && Z.ghost[K]) os = og = 0.0;   // ghost unknowns held at 0
    out[K] = os;
    out[Z.n + K] = og;
    acc.add(z[K] * os);
    acc.add(z[Z.n + K] * og);
  }
  if (part) {   // uniform over the grid: every thread reaches the barriers
    const CSum t = block_csum(acc, sh);
    if (threadIdx.x == 0) {
      part[2 * blockIdx.x] = t.hi;
      part[2 * blockIdx.x + 1] = t.lo;
    }
  }
}

// x = omega B^-1 b
__global__ void k_zsmooth_first(ZCells Z, double omega, const double* __restrict__ b,
                                double* __restrict__ x) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= Z.n) return;
  zfirst_sweep(Z, omega, b, (int32_t)K, x[K], x[Z.n + K]);
}

// the first two sweeps from zero in one pass: x1 = omega B^-1 b is formed
// wherever it is gathered, xo = x1 + omega B^-1 (b - J_z x1)
__global__ void __launch_bounds__(kT) k_zsmooth_two(ZCells Z, double omega,
                                                    const double* __restrict__ b,
                                                    double* __restrict__ xo) {
  const int64_t K = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (K >= Z.n) return;
  double os, og;
  zapply_cell_v(
      Z, [&](int32_t M, double& sv, double& gv) { zfirst_sweep(Z, omega, b, M, sv, gv); }, K,
      os, og);
  double xs, xg;
  zfirst_sweep(Z, omega, b, (int32_t)K, xs, xg);
  const double bs = b[K], bg = b[Z.n + K];
  const double rs = bs - os, rg = bg - og;
  xo[K] = xs + omega * (Z.bi[3 * K] * rs + Z.bi[3 * K + 1] * rg);
  xo[Z.n + K] = xg + omega * (Z.bi[3 * K + 1] * rs + Z.bi[3 * K + 2] * rg);
}

// xo = xi + omega B^-1 (b - J_z xi); with `part`, also the compensated
// block sums of b . xo (as k_zop)
__global__ void __launch_bounds__(kT) k_zsmooth(ZCells Z, double omega,
                                                const double* __restrict__ b,
                                                const double* __restrict__ xi,
                                                double* __restrict__ xo,
                                                double* __restrict__ part) {
  __shared__ double sh[32];
  const int64_t K = (int64_t)blockIdx.x * kT + threadIdx.x;
  CSum acc;
  if (K < Z.n) {
    double os, og;
    zapply_cell(Z, xi, xi + Z.n, K, os, og);
    const double bs = b[K], bg = b[Z.n + K];
    const double rs = bs - os, rg = bg - og;
    const double ys = xi[K] + omega * (Z.bi[3 * K] * rs + Z.bi[3 * K + 1] * rg);
    const double yg = xi[Z.n + K] + omega * (Z.bi[3 * K + 1] * rs + Z.bi[3 * K + 2] * rg);
    xo[K] = ys;
    xo[Z.n + K] = yg;
    acc.add(bs * ys);
    acc.add(bg * yg);
  }
  if (part) {
    const CSum t = block_csum(acc, sh);
    if (threadIdx.x == 0) {
      part[2 * blockIdx.x] = t.hi;
      part[2 * blockIdx.x + 1] = t.lo;
    }
  }
}

// r = b - J_z x
__global__ void __launch_bounds__(kT) k_zresid(ZCells Z, const double* __restrict__ b,
                                               const double* __restrict__ x,
                                               double* __restrict__ r) {
  const int64_t K = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (K >= Z.n) return;
  double os, og;
  zapply_cell(Z, x, x + Z.n, K, os, og);
  const bool gh = Z.ghost && Z.ghost[K];
  r[K] = gh ? 0.0 : b[K] - os;
  r[Z.n + K] = gh ? 0.0 : b[Z.n + K] - og;
}

// coarse (cell) residual: y-space residual of the rows attached to M and
// of column M, with r_row = r_s / 2 + r_g and r_col = r_s / 2 - r_g
// (also the first Jacobi sweep of the cell level from zero, x1 = sdc bc)
__global__ void k_zrestrict(const int32_t* __restrict__ mptr, const int32_t* __restrict__ mem,
                            const double* __restrict__ r, int64_t n, const double* __restrict__ sdc,
                            double* __restrict__ bc, double* __restrict__ x1) {
  const int64_t M = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (M >= n) return;
  double acc = 0;
  for (int32_t q = mptr[M]; q < mptr[M + 1]; ++q) {
    const int32_t p = mem[q];
    if (p < (int32_t)n)
      acc += 0.5 * r[p] + r[n + p];
    else
      acc += 0.5 * r[p - n] - r[p];   // r[n + (p - n)] is the g part of cell p - n
  }
  bc[M] = acc;
  x1[M] = sdc[M] * acc;
}

// x += P e: row K takes e[best K], column K takes e[K]
__global__ void k_zprolong(const int32_t* __restrict__ best, const double* __restrict__ e,
                           const uint8_t* __restrict__ ghost, int64_t n,
                           double* __restrict__ x) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= n || (ghost && ghost[K])) return;
  const double er = e[best[K]], ec = e[K];
  x[K] += 0.5 * (er + ec);
  x[n + K] += er - ec;
}

struct ZPrecond {
  ZCells Z;
  Hierarchy* H;
  double omega = 0.7;
  int pre = 2, post = 2;
  int64_t fuse_max = kZsmoothTwoMaxCells;   // the first two sweeps in one pass up to this size
  double *x, *x2, *res;   // 2n work vectors
};

// z = M r: block-Jacobi smoothing in (s, g), coarse correction through
// the cell hierarchy, block-Jacobi smoothing (symmetric).  With `part`
// (and at least one post-sweep) the last sweep also leaves the block sums
// of r . z there; returns whether it did.
static bool zprecondition(ZPrecond& P, const double* r, double* z, hipStream_t s,
                          double* part = nullptr) {
  const int64_t n = P.Z.n;
  const unsigned gb = blocks_for(n, kT);
  double* x = P.x;
  double* x2 = P.x2;
  int k0 = 1;
  // one pass for the first two sweeps saves a launch where launches cost
  // (up to ~10^6 cells); beyond, its wider gathers (b and B^-1 of every
  // neighbour instead of its iterate) cost more than the pass it saves
  if (P.pre >= 2 && n <= P.fuse_max) {
    ::bchar::ProfScope ps_("k_zsmooth_two", s);
    k_zsmooth_two<<<gb, kT, 0, s>>>(P.Z, P.omega, r, x);
    k0 = 2;
  } else {
    ::bchar::ProfScope ps_("k_zsmooth_first", s);
    k_zsmooth_first<<<gb, kT, 0, s>>>(P.Z, P.omega, r, x);
  }
  for (int k = k0; k < P.pre; ++k) {
    {
      ::bchar::ProfScope ps_("k_zsmooth", s);
      k_zsmooth<<<gb, kT, 0, s>>>(P.Z, P.omega, r, x, x2, nullptr);
    }
    std::swap(x, x2);
  }
  {
    ::bchar::ProfScope ps_("k_zresid", s);
    k_zresid<<<gb, kT, 0, s>>>(P.Z, r, x, P.res);
  }
  Level& L0 = P.H->lv[0];
  Level& L1 = P.H->lv[1];
  {
    ::bchar::ProfScope ps_("k_zrestrict", s);
    k_zrestrict<<<blocks_for(n, kT), kT, 0, s>>>(L0.mptr, L0.mem, P.res, n, L1.sdinv, L1.b,
                                                  L1.x2);
  }
  vcycle(*P.H, 1, s);
  {
    ::bchar::ProfScope ps_("k_zprolong", s);
    k_zprolong<<<gb, kT, 0, s>>>(P.Z.best, L1.x, P.Z.ghost, n, x);
  }
  for (int k = 0; k < P.post; ++k) {
    double* out = (k + 1 == P.post) ? z : x2;
    {
      ::bchar::ProfScope ps_("k_zsmooth", s);
      k_zsmooth<<<gb, kT, 0, s>>>(P.Z, P.omega, r, x, out, out == z ? part : nullptr);
    }
    if (out == x2) std::swap(x, x2);
  }
  if (P.post == 0)
    BCHAR_HIP(hipMemcpyAsync(z, x, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, s));
  BCHAR_HIP(hipGetLastError());
  return part != nullptr && P.post > 0;
}

// ====================================================================== Newton kernels

struct QpArrays {
  int64_t n, nnz;
  const int32_t *rptr, *col;        // CSR
  const int32_t *cptr, *crow, *cpos;  // CSC
  double *a;      // scaled A^(N), CSR order
  double *ac;     // CSC order
  double *rr, *ss;  // targets of sum a x (rows, cols)
  double *t, *dt;   // per entry
  double *F;        // 2n residual
};

__global__ void k_gather_q(const double* __restrict__ src, const int32_t* __restrict__ idx,
                           int64_t n, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = src[idx[e]];
}

__global__ void k_scale_a(const double* __restrict__ an, double inv, int64_t nnz,
                          double* __restrict__ a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) a[k] = an[k] * inv;
}

// rr[i] = b_row_i/scale - sum_row a ; ss[j] = b_j/scale - sum_col a
__global__ void k_targets(const int32_t* __restrict__ rptr, const int32_t* __restrict__ cptr,
                          const double* __restrict__ a, const double* __restrict__ ac,
                          const double* __restrict__ b_row, const double* __restrict__ b,
                          double inv, int64_t n, double* __restrict__ rr,
                          double* __restrict__ ss) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  CSum r, c;
  r.add(b_row[i] * inv);
  for (int32_t k = rptr[i]; k < rptr[i + 1]; ++k) r.add(-a[k]);
  c.add(b[i] * inv);
  for (int32_t e = cptr[i]; e < cptr[i + 1]; ++e) c.add(-ac[e]);
  rr[i] = r.value();
  ss[i] = c.value();
}

__device__ __forceinline__ double clipv(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// F = [sum_row a clip(t + step dt) - rr ; sum_col ... - ss]
__global__ void k_residual(const int32_t* __restrict__ rptr, const int32_t* __restrict__ cptr,
                           const int32_t* __restrict__ cpos, const double* __restrict__ a,
                           const double* __restrict__ ac, const double* __restrict__ t,
                           const double* __restrict__ dt, double step, double lo, double hi,
                           const double* __restrict__ rr, const double* __restrict__ ss,
                           int64_t n, double* __restrict__ F) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  CSum r, c;
  r.add(-rr[i]);
  for (int32_t k = rptr[i]; k < rptr[i + 1]; ++k) {
    const double tk = dt ? t[k] + step * dt[k] : t[k];
    r.add(a[k] * clipv(tk, lo, hi));
  }
  c.add(-ss[i]);
  for (int32_t e = cptr[i]; e < cptr[i + 1]; ++e) {
    const int32_t k = cpos[e];
    const double tk = dt ? t[k] + step * dt[k] : t[k];
    c.add(ac[e] * clipv(tk, lo, hi));
  }
  F[i] = r.value();
  F[n + i] = c.value();
}

// fine bipartite weights a_k^2 * free_k in graph order: row part is CSR
// order, column part is CSC order.  An entry counts as free within `band`
// outside the box as well: entries at a kink (zero multiplier on an active
// bound) then keep their cells coupled instead of splitting them into
// pieces whose multipliers the Newton step would move without bound.
__global__ void k_fine_weights(const double* __restrict__ a, const int32_t* __restrict__ cpos,
                               const double* __restrict__ t, double lo, double hi, double band,
                               int64_t nnz, double* __restrict__ w) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const double tk = t[k];
  w[k] = (tk > lo - band && tk < hi + band) ? a[k] * a[k] : 0.0;
  const int32_t kp = cpos[k];
  const double tp = t[kp];
  w[nnz + k] = (tp > lo - band && tp < hi + band) ? a[kp] * a[kp] : 0.0;
}

__global__ void k_fine_graph(const int32_t* __restrict__ rptr, const int32_t* __restrict__ col,
                             const int32_t* __restrict__ cptr, const int32_t* __restrict__ crow,
                             int64_t n, int64_t nnz, int32_t* __restrict__ gptr,
                             int32_t* __restrict__ gnbr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    gptr[i] = rptr[i];
    gptr[n + i] = (int32_t)nnz + cptr[i];
    for (int32_t k = rptr[i]; k < rptr[i + 1]; ++k) gnbr[k] = (int32_t)n + col[k];
    for (int32_t e = cptr[i]; e < cptr[i + 1]; ++e) gnbr[nnz + e] = crow[e];
  }
  if (i == 0) gptr[2 * n] = (int32_t)(2 * nnz);
}

// (s, g) right-hand side from F: fr = -F_row, fc = F_col;
// b_s = fr + fc, b_g = (fr - fc) / 2
__global__ void k_zrhs(const double* __restrict__ F, int64_t n, double* __restrict__ bz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double fr = -F[i], fc = F[n + i];
    bz[i] = fr + fc;
    bz[n + i] = 0.5 * (fr - fc);
  }
}

// A pattern of several connected components leaves one null direction of
// the Newton matrix per component (its multipliers moved by a constant):
// the right-hand side is made orthogonal to each.  In y = (mu, -nu)
// coordinates node v carries -F_row (rows) or F_col (columns); dm[c] =
// their mean over component c (one wave per label, members in node order).
__global__ void __launch_bounds__(64) k_group_mean(int64_t n, const int32_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ perm,
                                                   const double* __restrict__ F,
                                                   double* __restrict__ dm) {
  const int64_t c = blockIdx.x;
  const int32_t p0 = ptr[c], p1 = ptr[c + 1];
  if (p0 == p1) return;
  CSum acc;
  for (int32_t q = p0 + (int32_t)threadIdx.x; q < p1; q += 64) {
    const int64_t v = perm[q];
    acc.add(v < n ? -F[v] : F[v]);
  }
  wave_csum(acc);
  if (threadIdx.x == 0) dm[c] = acc.value() / (double)(p1 - p0);
}

// the (s, g) right-hand side of the mean-free y right-hand side
__global__ void k_group_fix(int64_t n, const int32_t* __restrict__ lab,
                            const double* __restrict__ dm, double* __restrict__ bz) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= n) return;
  const double dr = dm[lab[K]], dc = dm[lab[n + K]];
  bz[K] -= dr + dc;
  bz[n + K] -= 0.5 * (dr - dc);
}

// residuals of ghost cells' rows and columns (no target) set to 0
__global__ void k_zero_ghost(const uint8_t* __restrict__ ghost, int64_t n,
                             double* __restrict__ F) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K < n && ghost[K]) {
    F[K] = 0.0;
    F[n + K] = 0.0;
  }
}

__global__ void k_sub_scalar(double* __restrict__ v, const double* __restrict__ sum,
                             double inv_n, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] -= sum[0] * inv_n;
}

// CG vector updates (x += alpha p, r -= alpha q; p = z + beta p) with the
// scalar they need summed from the block partials of the kernel before
// (k_zop: p.q; the preconditioner's last sweep: r.z) inside the kernel:
// every block sums all partials exactly as k_reduce_final_sum does (the
// same bits), so no launch sits between.  A
// grid of at most kCgBlocks blocks (grid-stride) keeps the repeated reads
// of the partials small.
constexpr int kCgBlocks = 512;

__global__ void __launch_bounds__(kFinalThreads) k_cg_update_part(
    const double* __restrict__ rz, const double* __restrict__ part, int np, int64_t n,
    double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
    const double* __restrict__ q) {
  __shared__ double sh[32];
  const double pq = block_final_sum(part, np, sh);
  const double alpha = pq != 0.0 ? *rz / pq : 0.0;
  const int64_t stride = (int64_t)gridDim.x * kFinalThreads;
  for (int64_t i = (int64_t)blockIdx.x * kFinalThreads + threadIdx.x; i < n; i += stride) {
    x[i] += alpha * p[i];
    r[i] -= alpha * q[i];
  }
}

// also stores the new r.z (block 0) for the next update
__global__ void __launch_bounds__(kFinalThreads) k_cg_dir_part(
    const double* __restrict__ rz_old, const double* __restrict__ part, int np,
    double* __restrict__ rz_new, int64_t n, const double* __restrict__ z,
    double* __restrict__ p) {
  __shared__ double sh[32];
  const double rzn = block_final_sum(part, np, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) *rz_new = rzn;
  const double beta = *rz_old != 0.0 ? rzn / *rz_old : 0.0;
  const int64_t stride = (int64_t)gridDim.x * kFinalThreads;
  for (int64_t i = (int64_t)blockIdx.x * kFinalThreads + threadIdx.x; i < n; i += stride)
    p[i] = z[i] + beta * p[i];
}

// p = z + (rz_new / rz_old) p
__global__ void k_cg_dir(const double* __restrict__ rz_old, const double* __restrict__ rz_new,
                         int64_t n, const double* __restrict__ z, double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double beta = *rz_old != 0.0 ? *rz_new / *rz_old : 0.0;
  p[i] = z[i] + beta * p[i];
}

// dual direction from the (s, g) solution (mean of s removed) and the
// per-entry increments of t
__global__ void k_zdual_dir(const int32_t* __restrict__ rptr, const int32_t* __restrict__ col,
                            const double* __restrict__ a, const double* __restrict__ z,
                            const double* __restrict__ ssum, double inv_n, int64_t n,
                            double* __restrict__ dmu, double* __restrict__ dnu,
                            double* __restrict__ dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double si = z[i] - ssum[0] * inv_n;
  const double gi = z[n + i];
  dmu[i] = si + 0.5 * gi;
  dnu[i] = -(si - 0.5 * gi);
  for (int32_t k = rptr[i]; k < rptr[i + 1]; ++k) {
    const int32_t j = col[k];
    dt[k] = a[k] * (j == (int32_t)i ? gi : (z[i] - z[j]) + 0.5 * (gi + z[n + j]));
  }
}

// derivative of the dual function along the direction, at y + step d:
// sum over cells of dmu_i F_i + dnu_i G_i with the row and column residuals
// F_i, G_i of t + step dt formed cell by cell (each is small near the
// solution, so the sum does not cancel the large terms of sum_k x_k dt_k
// against d . (r; s))
__global__ void __launch_bounds__(kT) k_dphi_part(
    const int32_t* __restrict__ rptr, const int32_t* __restrict__ cptr,
    const int32_t* __restrict__ cpos, const double* __restrict__ a,
    const double* __restrict__ ac, const double* __restrict__ t, const double* __restrict__ dt,
    double step, double lo, double hi, const double* __restrict__ rr,
    const double* __restrict__ ss, const double* __restrict__ dmu,
    const double* __restrict__ dnu, int64_t n, double* __restrict__ part) {
  __shared__ double sh[32];
  CSum acc;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kT) {
    CSum r, c;
    r.add(-rr[i]);
    for (int32_t k = rptr[i]; k < rptr[i + 1]; ++k)
      r.add(a[k] * clipv(t[k] + step * dt[k], lo, hi));
    c.add(-ss[i]);
    for (int32_t e = cptr[i]; e < cptr[i + 1]; ++e) {
      const int32_t k = cpos[e];
      c.add(ac[e] * clipv(t[k] + step * dt[k], lo, hi));
    }
    acc.add(dmu[i] * r.value());
    acc.add(dnu[i] * c.value());
  }
  CSum tot = block_csum(acc, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = tot.hi;
    part[2 * blockIdx.x + 1] = tot.lo;
  }
}

// t_k from per-cell multipliers z = (s, g): a_k g_K on the diagonal entry
// of cell K, a_k ((s_K - s_M) + (g_K + g_M) / 2) elsewhere
__global__ void k_t_from_z(const int32_t* __restrict__ rptr, const int32_t* __restrict__ col,
                           const double* __restrict__ a, const double* __restrict__ z, int64_t n,
                           double* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double si = z[i], gi = z[n + i];
  for (int32_t k = rptr[i]; k < rptr[i + 1]; ++k) {
    const int32_t j = col[k];
    t[k] = a[k] * (j == (int32_t)i ? gi : (si - z[j]) + 0.5 * (gi + z[n + j]));
  }
}

// z += step * (solution with the mean of its s part removed), summed with
// compensation: z holds the leading parts of the 2n multipliers and, from
// z + 2n on, what their rounding lost (cells that barely move carry
// multipliers of 1e9 and more, whose increments would otherwise drift from
// the increments of t by units in their last place)
__global__ void k_zdual_acc(const double* __restrict__ sol, const double* __restrict__ ssum,
                            double inv_n, double step, int64_t n, double* __restrict__ z) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // the increment step * (sol - mean) as p + pe + step * ve, exactly but
  // for the last product, and its sum with z by TwoSum
  double v, ve, hi, err;
  two_sum(sol[i], -(ssum[0] * inv_n), v, ve);
  double p = step * v, pe = fma(step, v, -p);
  two_sum(z[i], p, hi, err);
  z[i] = hi;
  z[2 * n + i] += (err + pe) + step * ve;
  p = step * sol[n + i];
  pe = fma(step, sol[n + i], -p);
  two_sum(z[n + i], p, hi, err);
  z[n + i] = hi;
  z[3 * n + i] += err + pe;
}

// mu = s + g/2, nu = -(s - g/2)
__global__ void k_mu_nu(const double* __restrict__ z, int64_t n, double* __restrict__ mu,
                        double* __restrict__ nu) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  mu[i] = z[i] + 0.5 * z[n + i];
  nu[i] = -(z[i] - 0.5 * z[n + i]);
}

__global__ void k_axpy2(double* __restrict__ y, const double* __restrict__ x, double s,
                        int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += s * x[i];
}

// x = clip(t) (semismooth answer) or the interior point's x (xi non-null);
// counts the entries within `thr` of each bound
__global__ void k_final(const double* __restrict__ an, const double* __restrict__ t,
                        const double* __restrict__ xi, double lo, double hi, double thr,
                        int clip, int64_t nnz, double* __restrict__ x, double* __restrict__ A,
                        int32_t* __restrict__ counts) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  // the interior point's iterate stays in the box up to its rounding; a
  // corrected one is taken as it is (clip = 0)
  const double v = xi ? xi[k] : t[k];
  const double xk = clip ? clipv(v, lo, hi) : v;
  x[k] = xk;
  A[k] = an[k] * (1.0 + xk);
  if (xk - lo <= thr) atomicAdd(&counts[0], 1);
  if (hi - xk <= thr) atomicAdd(&counts[1], 1);
}

// ====================================================================== interior point
//
// Primal-dual interior-point iteration (Mehrotra predictor-corrector) on
//   min 1/2 x^T x,  sum_row a x = rr,  sum_col a x = ss,  lo <= x <= hi,
// with slacks sl = x - lo, su = hi - x and bound multipliers zl, zu >= 0.
// Eliminating dx = D (B^T dy + h), D = 1 / (1 + zl / sl + zu / su), leaves
// the normal equations B D B^T dy = -(B (x + D h) - r): the weighted
// bipartite Laplacian of the Newton systems with weights a_k^2 D_k, all
// positive, solved by the same preconditioned CG.  B^T dy = dt is the
// change of t, carried per entry as in the semismooth iteration, so that
// the interior point's t seeds it.

struct IpmArrays {
  double *x, *sl, *su, *zl, *zu;   // iterate
  double *D, *h, *dxa;             // scaling, right-hand side, predictor dx
  double *dx, *dzl, *dzu;          // step
  double lo, hi;
  int has_hi;                      // level 0: both bounds; level 1: lower only
};

// Crossover from an interior point: the side of every entry, -1 on the
// lower bound (its slack below `ratio` times its multiplier), +1 on the
// upper bound, 0 free (degenerate entries, slack and multiplier alike
// small, stay free).
__global__ void k_xover_state(IpmArrays I, double ratio, int64_t nnz,
                              int8_t* __restrict__ side) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  int8_t v = 0;
  if (I.sl[k] < ratio * I.zl[k])
    v = -1;
  else if (I.has_hi && I.su[k] < ratio * I.zu[k])
    v = 1;
  side[k] = v;
}

// Sides read off the multipliers (a primal-dual active-set update): an
// entry whose t lies below the lower bound is pinned there, above the upper
// bound pinned there, and free otherwise.
__global__ void k_side_from_t(const double* __restrict__ t, double lo, double hi, int64_t nnz,
                              int8_t* __restrict__ side) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const double v = t[k];
  side[k] = v < lo ? (int8_t)-1 : (v > hi ? (int8_t)1 : (int8_t)0);
}

// Residual with the sides fixed: x_k is the bound of a pinned entry and
// t_k of a free one (k_residual with clip replaced by the sides).
__global__ void k_residual_sides(const int32_t* __restrict__ rptr, const int32_t* __restrict__ cptr,
                                 const int32_t* __restrict__ cpos, const double* __restrict__ a,
                                 const double* __restrict__ ac, const double* __restrict__ t,
                                 const int8_t* __restrict__ side, double lo, double hi,
                                 const double* __restrict__ rr, const double* __restrict__ ss,
                                 int64_t n, double* __restrict__ F) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  CSum r, c;
  r.add(-rr[i]);
  for (int32_t k = rptr[i]; k < rptr[i + 1]; ++k) {
    const double xk = side[k] < 0 ? lo : (side[k] > 0 ? hi : t[k]);
    r.add(a[k] * xk);
  }
  c.add(-ss[i]);
  for (int32_t e = cptr[i]; e < cptr[i + 1]; ++e) {
    const int32_t k = cpos[e];
    const double xk = side[k] < 0 ? lo : (side[k] > 0 ? hi : t[k]);
    c.add(ac[e] * xk);
  }
  F[i] = r.value();
  F[n + i] = c.value();
}

// fine weights a_k^2 on the free entries (graph order, as k_fine_weights)
__global__ void k_side_weights(const double* __restrict__ a, const int32_t* __restrict__ cpos,
                               const int8_t* __restrict__ side, int64_t nnz,
                               double* __restrict__ w) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  w[k] = side[k] == 0 ? a[k] * a[k] : 0.0;
  const int32_t kp = cpos[k];
  w[nnz + k] = side[kp] == 0 ? a[kp] * a[kp] : 0.0;
}

// D and the per-block complementarity sums sl zl + su zu
__global__ void __launch_bounds__(kT) k_ipm_prep(IpmArrays I, int64_t nnz,
                                                 double* __restrict__ part) {
  __shared__ double sh[32];
  CSum acc;
  for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * kT) {
    const double sl = I.sl[k], zl = I.zl[k];
    double sig = zl / sl;
    acc.add(sl * zl);
    if (I.has_hi) {
      const double su = I.su[k], zu = I.zu[k];
      sig += zu / su;
      acc.add(su * zu);
    }
    I.D[k] = 1.0 / (1.0 + sig);
  }
  CSum r = block_csum(acc, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r.hi;
    part[2 * blockIdx.x + 1] = r.lo;
  }
}

// complementarity targets: sl dzl + zl dx = cl, su dzu - zu dx = cu.
// Predictor: cl = -sl zl, cu = -su zu.  Corrector: sigma mu minus those
// and the predictor's second-order terms.
struct IpmTargets {
  double cl, cu;
};
__device__ __forceinline__ IpmTargets ipm_targets(const IpmArrays& I, int64_t k, int corr,
                                                  double smu) {
  const double sl = I.sl[k], zl = I.zl[k];
  IpmTargets c;
  c.cu = 0.0;
  if (!corr) {
    c.cl = -sl * zl;
    if (I.has_hi) c.cu = -I.su[k] * I.zu[k];
  } else {
    const double dxa = I.dxa[k];
    const double dzla = -zl - zl * dxa / sl;
    c.cl = smu - sl * zl - dxa * dzla;
    if (I.has_hi) {
      const double su = I.su[k], zu = I.zu[k];
      const double dzua = -zu + zu * dxa / su;
      c.cu = smu - su * zu + dxa * dzua;
    }
  }
  return c;
}

// h = -(x - t - zl + zu) + cl / sl - cu / su
__global__ void k_ipm_h(IpmArrays I, const double* __restrict__ t, int corr, double smu,
                        int64_t nnz) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const IpmTargets c = ipm_targets(I, k, corr, smu);
  double h = t[k] - I.x[k] + I.zl[k] + c.cl / I.sl[k];
  if (I.has_hi) h += -I.zu[k] - c.cu / I.su[k];
  I.h[k] = h;
}

// fine weights a_k^2 D_k in graph order (CSR part, CSC part)
__global__ void k_ipm_weights(const double* __restrict__ a, const int32_t* __restrict__ cpos,
                              const double* __restrict__ D, int64_t nnz,
                              double* __restrict__ w) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  w[k] = (a[k] * a[k]) * D[k];
  const int32_t kp = cpos[k];
  w[nnz + k] = (a[kp] * a[kp]) * D[kp];
}

// per cell: rp = B x - r and fv = B (x + D h) - r (row part, then column part)
__global__ void k_ipm_rhs(const int32_t* __restrict__ rptr, const int32_t* __restrict__ cptr,
                          const int32_t* __restrict__ cpos, const double* __restrict__ a,
                          const double* __restrict__ ac, IpmArrays I,
                          const double* __restrict__ rr, const double* __restrict__ ss,
                          int64_t n, double* __restrict__ rp, double* __restrict__ fv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  CSum r0, r1, c0, c1;
  r0.add(-rr[i]);
  r1.add(-rr[i]);
  for (int32_t k = rptr[i]; k < rptr[i + 1]; ++k) {
    r0.add(a[k] * I.x[k]);
    r1.add(a[k] * I.x[k]);
    r1.add(a[k] * (I.D[k] * I.h[k]));
  }
  c0.add(-ss[i]);
  c1.add(-ss[i]);
  for (int32_t e = cptr[i]; e < cptr[i + 1]; ++e) {
    const int32_t k = cpos[e];
    c0.add(ac[e] * I.x[k]);
    c1.add(ac[e] * I.x[k]);
    c1.add(ac[e] * (I.D[k] * I.h[k]));
  }
  rp[i] = r0.value();
  rp[n + i] = c0.value();
  fv[i] = r1.value();
  fv[n + i] = c1.value();
}

// step from dt = B^T dy: dx, dzl, dzu, and per block the largest inverse
// step to the boundary, max(-dx / sl, dx / su) and max(-dzl / zl, -dzu / zu)
__global__ void __launch_bounds__(kT) k_ipm_dir(IpmArrays I, const double* __restrict__ dt,
                                                int corr, double smu, int64_t nnz,
                                                double* __restrict__ part) {
  __shared__ double sh[16];
  double ip = 0.0, id = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * kT) {
    const IpmTargets c = ipm_targets(I, k, corr, smu);
    const double sl = I.sl[k], zl = I.zl[k];
    const double dx = I.D[k] * (dt[k] + I.h[k]);
    const double dzl = (c.cl - zl * dx) / sl;
    I.dx[k] = dx;
    I.dzl[k] = dzl;
    if (!corr) I.dxa[k] = dx;
    ip = fmax(ip, -dx / sl);
    id = fmax(id, -dzl / zl);
    if (I.has_hi) {
      const double su = I.su[k], zu = I.zu[k];
      const double dzu = (c.cu + zu * dx) / su;
      I.dzu[k] = dzu;
      ip = fmax(ip, dx / su);
      id = fmax(id, -dzu / zu);
    }
  }
  ip = block_max(ip, sh);
  __syncthreads();
  id = block_max(id, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = ip;
    part[kRedBlocks + blockIdx.x] = id;
  }
}

// complementarity after the predictor step (ap, ad), per block
__global__ void __launch_bounds__(kT) k_ipm_muaff(IpmArrays I, double ap, double ad,
                                                  int64_t nnz, double* __restrict__ part) {
  __shared__ double sh[32];
  CSum acc;
  for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * kT) {
    const double dx = I.dx[k];
    acc.add((I.sl[k] + ap * dx) * (I.zl[k] + ad * I.dzl[k]));
    if (I.has_hi) acc.add((I.su[k] - ap * dx) * (I.zu[k] + ad * I.dzu[k]));
  }
  CSum r = block_csum(acc, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r.hi;
    part[2 * blockIdx.x + 1] = r.lo;
  }
}

__global__ void k_ipm_update(IpmArrays I, double* __restrict__ t, const double* __restrict__ dt,
                             double ap, double ad, int64_t nnz) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const double dx = I.dx[k];
  I.x[k] += ap * dx;
  I.sl[k] += ap * dx;
  I.zl[k] += ad * I.dzl[k];
  if (I.has_hi) {
    I.su[k] -= ap * dx;
    I.zu[k] += ad * I.dzu[k];
  }
  t[k] += ad * dt[k];
}

// Warm start from multipliers: t = a (mu + nu) of the previous solve on
// this matrix.  x = t moved at least theta inside the box, zl = (x - t)+ +
// theta, zu = (t - x)+ + theta: dual feasible (x - t - zl + zu = 0) and
// every slack and multiplier at least theta.
__global__ void k_ipm_init_warm(IpmArrays I, const double* __restrict__ t, double theta,
                                int64_t nnz) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const double tk = t[k];
  double x = tk > I.lo + theta ? tk : I.lo + theta;
  if (I.has_hi) x = x < I.hi - theta ? x : I.hi - theta;
  I.x[k] = x;
  I.sl[k] = x - I.lo;
  I.zl[k] = (x > tk ? x - tk : 0.0) + theta;
  I.su[k] = I.has_hi ? I.hi - x : 1.0;
  I.zu[k] = I.has_hi ? (tk > x ? tk - x : 0.0) + theta : 0.0;
}

__global__ void k_ipm_init(IpmArrays I, int64_t nnz) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  I.x[k] = 0.0;
  I.sl[k] = -I.lo;
  I.zl[k] = 1.0;
  I.su[k] = I.has_hi ? I.hi : 1.0;
  I.zu[k] = I.has_hi ? 1.0 : 0.0;
}

// ====================================================================== solver

bchar_status solve_qp(const bchar_mesh_s* m, const int32_t* row_ptr, const int32_t* col,
                      const Csc& csc, const double* AN, const double* b_row,
                      const Groups* groups, int64_t nnz, const bchar_opts& o, double* x_out,
                      double* mu_out, double* nu_out, double* A_out, double* zdual,
                      int warm_level, int& warm_newton_skip, QpResult& res, Arena& ws,
                      hipStream_t s) {
  const int64_t n = m->n_cells;
  const int64_t n2 = 2 * n;
  const double scale = m->bmax;
  const double inv = 1.0 / scale;
  const unsigned gn = blocks_for(n, kT), gn2 = blocks_for(n2, kT), gz = blocks_for(nnz, kT);

  Reducer red{ws.get<double>(2 * kRedBlocks + 2), ws.get<double>(16), s};
  double* zpart = ws.get<double>(2 * (size_t)blocks_for(n, kT) + 2);   // block sums
  double* gmean = groups ? ws.get<double>(n2) : nullptr;   // per-component means
  double* zsave = ws.get<double>(4 * (size_t)n + 1);   // interior-point multipliers
  double* tsave = ws.get<double>((size_t)nnz + 1);

  QpArrays Q{};
  Q.n = n;
  Q.nnz = nnz;
  Q.rptr = row_ptr;
  Q.col = col;
  Q.cptr = csc.ptr;
  Q.crow = csc.row;
  Q.cpos = csc.pos;
  Q.a = ws.get<double>(nnz + 1);
  Q.ac = ws.get<double>(nnz + 1);
  Q.rr = ws.get<double>(n);
  Q.ss = ws.get<double>(n);
  Q.t = ws.get<double>(nnz + 1);
  Q.dt = ws.get<double>(nnz + 1);
  Q.F = ws.get<double>(n2);
  double* dmu = ws.get<double>(n);
  double* dnu = ws.get<double>(n);
  {
    ::bchar::ProfScope ps_("k_scale_a", s);
    k_scale_a<<<gz, kT, 0, s>>>(AN, inv, nnz, Q.a);
  }
  {
    ::bchar::ProfScope ps_("k_gather_q", s);
    k_gather_q<<<gz, kT, 0, s>>>(Q.a, csc.pos, nnz, Q.ac);
  }
  {
    ::bchar::ProfScope ps_("k_targets", s);
    k_targets<<<gn, kT, 0, s>>>(row_ptr, csc.ptr, Q.a, Q.ac, b_row, m->b.as<double>(), inv, n,
                                Q.rr, Q.ss);
  }
  BCHAR_HIP(hipGetLastError());

  // bipartite graph (y space) and the cell hierarchy, pattern from a^2
  Level fine;
  fine.n = n2;
  fine.ne = 2 * nnz;
  fine.ptr = ws.get<int32_t>(n2 + 1);
  fine.nbr = ws.get<int32_t>(2 * nnz + 1);
  fine.w = ws.get<double>(2 * nnz + 1);
  fine.w0 = ws.get<double>(2 * nnz + 1);
  {
    ::bchar::ProfScope ps_("k_fine_graph", s);
    k_fine_graph<<<gn, kT, 0, s>>>(row_ptr, col, csc.ptr, csc.row, n, nnz, fine.ptr, fine.nbr);
  }
  fill_f64(Q.t, 0.0, nnz, s);
  {
    ::bchar::ProfScope ps_("k_fine_weights", s);
    k_fine_weights<<<gz, kT, 0, s>>>(Q.a, csc.pos, Q.t, -HUGE_VAL, HUGE_VAL, 0.0, nnz, fine.w0);
  }
  BCHAR_HIP(hipGetLastError());
  double dmax = 0;
  {
    double* dtmp = ws.get<double>(n2);
    double* stmp = ws.get<double>(n2);
    {
      ::bchar::ProfScope ps_("k_level_diag", s);
      k_level_diag<<<gn2, kT, 0, s>>>(fine.ptr, fine.w0, nullptr, n2, 0.0, 1.0, 0, dtmp, stmp);
    }
    red.maxabs(dtmp, n2, 0);
    dmax = red.fetch(0);
  }
  Hierarchy H;
  H.skip = o.cycle_skip ? 1 : 0;
  const double th0 = trace_enabled() ? wall_seconds() : 0.0;
  build_hierarchy(H, fine, row_ptr, col, Q.a, n, ws, s);
  if (trace_enabled()) {
    BCHAR_HIP(hipStreamSynchronize(s));
    fprintf(stderr, "[bchar] hierarchy: %zu levels in %.3f ms:", H.lv.size(),
            1e3 * (wall_seconds() - th0));
    for (auto& L : H.lv) fprintf(stderr, " %lld/%lld", (long long)L.n, (long long)L.ne);
    fprintf(stderr, "\n");
  }
  Level& L0 = H.lv[0];

  ZPrecond P;
  P.H = &H;
  P.fuse_max = o.z_fuse_max_cells;
  P.Z.n = n;
  P.Z.rptr = row_ptr;
  P.Z.col = col;
  P.Z.cptr = csc.ptr;
  P.Z.crow = csc.row;
  P.Z.cpos = csc.pos;
  int32_t* dpos = ws.get<int32_t>(n);
  {
    ::bchar::ProfScope ps_("k_diag_pos", s);
    k_diag_pos<<<gn, kT, 0, s>>>(row_ptr, col, n, dpos);
  }
  P.Z.dpos = dpos;
  P.Z.best = L0.agg;   // rows 0..n-1 of the level-0 aggregation
  P.Z.w = L0.w;
  P.Z.wc = L0.w + nnz;
  P.Z.tau_s = ws.get<double>(n);
  P.Z.tau_g = ws.get<double>(n);
  P.Z.bi = ws.get<double>(3 * n);
  P.Z.ghost = m->ghost.as<uint8_t>();
  // the constant-s direction is removed from every system unless ghost
  // cells (multipliers held at 0) anchor the multipliers
  const double inv_mean = P.Z.ghost ? 0.0 : 1.0 / (double)n;
  auto zero_ghost = [&](double* v) {
    if (!P.Z.ghost) return;
    ::bchar::ProfScope ps_("k_zero_ghost", s);
    k_zero_ghost<<<gn, kT, 0, s>>>(P.Z.ghost, n, v);
    BCHAR_HIP(hipGetLastError());
  };
  P.x = ws.get<double>(n2);
  P.x2 = ws.get<double>(n2);
  P.res = ws.get<double>(n2);

  double *cx = ws.get<double>(n2), *cr = ws.get<double>(n2), *cz = ws.get<double>(n2),
         *cp = ws.get<double>(n2), *cq = ws.get<double>(n2);

  const double tol = o.qp_tol;
  res = QpResult{};
  res.coarse_bytes = H.fused_bytes;
  res.smooth_bytes = H.smooth_bytes;

  // Newton matrix values: per-cell blocks and every level of the hierarchy,
  // from the fine weights in L0.w
  auto refresh = [&]() {
    {
      ::bchar::ProfScope ps_("k_zcells", s);
      k_zcells<<<gn, kT, 0, s>>>(P.Z, 1e-14, H.mu);
    }
    BCHAR_HIP(hipGetLastError());
    refresh_hierarchy(H, s);
  };

  // One CG iteration split after its update: the update half (product
  // J p, p.q, x/r update with r.z in rz) and units that run the next
  // iteration's preconditioner (r.z into rz_next), direction and update.
  const unsigned gcg = std::min<unsigned>(gn2, kCgBlocks);
  auto cg_update_half = [&](const double* rzc, hipStream_t st) {
    {
      ::bchar::ProfScope ps_("k_zop", st);
      k_zop<<<gn, kT, 0, st>>>(P.Z, cp, cq, zpart);
    }
    {
      ::bchar::ProfScope ps_("k_cg_update_part", st);
      k_cg_update_part<<<gcg, kFinalThreads, 0, st>>>(rzc, zpart, (int)gn, n2, cx, cr, cp, cq);
    }
    BCHAR_HIP(hipGetLastError());
  };
  // units, then (with `check`) the residual check's max |r| into out[11]
  auto cg_units = [&](int units, double* a, double* b, bool check, hipStream_t st) {
    Reducer rs = red;
    rs.s = st;
    for (int u = 0; u < units; ++u) {
      if (zprecondition(P, cr, cz, st, zpart)) {
        ::bchar::ProfScope ps_("k_cg_dir_part", st);
        k_cg_dir_part<<<gcg, kFinalThreads, 0, st>>>(a, zpart, (int)gn, b, n2, cz, cp);
      } else {
        rs.dot(cr, cz, n2, (int)(b - red.out));
        ::bchar::ProfScope ps_("k_cg_dir", st);
        k_cg_dir<<<gn2, kT, 0, st>>>(a, b, n2, cz, cp);
      }
      BCHAR_HIP(hipGetLastError());
      cg_update_half(b, st);
      std::swap(a, b);
    }
    if (check) rs.maxabs(cr, n2, 11);
  };
  // The iterations between two residual checks launch the same few dozen
  // kernels with the same arguments every time (the hierarchy's buffers
  // are fixed for the whole solve): they are captured once per solve and
  // replayed, one host launch per four iterations instead of a few dozen
  // (the step time is the same within noise: the idle time between these
  // short kernels is the device's own dependency gap).
  // Graph 0 holds the three units after iteration 0, graph 1 the four
  // between two later checks; each ends with the check's max |r|.
  // Capture runs on a stream of its own (the solve's stream may be the
  // null stream, which cannot be captured); the graphs replay on the
  // solve's stream.
  struct CgGraphs {
    hipStream_t ls = nullptr;   // replays go to this stream
    hipStream_t cs = nullptr;
    hipGraph_t g[2] = {nullptr, nullptr};
    hipGraphExec_t x[2] = {nullptr, nullptr};
    ~CgGraphs() {
      // (every replay is followed by a read of its check; this also covers
      // a replay an exception left behind)
      if (x[0] || x[1]) (void)hipStreamSynchronize(ls);
      for (int i = 0; i < 2; ++i) {
        if (x[i]) (void)hipGraphExecDestroy(x[i]);
        if (g[i]) (void)hipGraphDestroy(g[i]);
      }
      if (cs) (void)hipStreamDestroy(cs);
    }
  } G;
  G.ls = s;
  const bool graphs_ok = o.cg_graphs != 0;
  auto capture_units = [&](int which, int units, double* a, double* b) {
    ProfModeGuard g_(ProfMode::off);
    if (!G.cs) BCHAR_HIP(hipStreamCreateWithFlags(&G.cs, hipStreamNonBlocking));
    BCHAR_HIP(hipStreamBeginCapture(G.cs, hipStreamCaptureModeRelaxed));
    try {
      cg_units(units, a, b, true, G.cs);
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(G.cs, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    BCHAR_HIP(hipStreamEndCapture(G.cs, &G.g[which]));
    BCHAR_HIP(hipGraphInstantiateWithFlags(&G.x[which], G.g[which], 0));
  };

  // Preconditioned CG on J d = -fv (fv: row part, then column part), in
  // the per-cell coordinates with the constant-s direction removed.  Leaves
  // the per-cell solution in cx, the multiplier direction in dmu, dnu and
  // the entry increments a_k (dmu_K + dnu_M) in Q.dt; returns iterations.
  auto pcg = [&](const double* fv, double cg_tol, bool from_cx, int max_cg) -> int {
    {
      ::bchar::ProfScope ps_("k_zrhs", s);
      k_zrhs<<<gn, kT, 0, s>>>(fv, n, cr);
    }
    if (groups) {
      {
        ::bchar::ProfScope ps_("k_group_mean", s);
        k_group_mean<<<(unsigned)n2, 64, 0, s>>>(n, groups->ptr, groups->perm, fv, gmean);
      }
      {
        ::bchar::ProfScope ps_("k_group_fix", s);
        k_group_fix<<<gn, kT, 0, s>>>(n, groups->lab, gmean, cr);
      }
      BCHAR_HIP(hipGetLastError());
    }
    red.sum(cr, n, 12);
    {
      ::bchar::ProfScope ps_("k_sub_scalar", s);
      k_sub_scalar<<<gn, kT, 0, s>>>(cr, red.out + 12, inv_mean, n);
    }
    if (from_cx) {
      // start from the solution already in cx: r = rhs - J cx
      {
        ::bchar::ProfScope ps_("k_zop", s);
        k_zop<<<gn, kT, 0, s>>>(P.Z, cx, cq, nullptr);
      }
      {
        ::bchar::ProfScope ps_("k_axpy2", s);
        k_axpy2<<<gn2, kT, 0, s>>>(cr, cq, -1.0, n2);
      }
    } else {
      fill_f64(cx, 0.0, n2, s);
    }
    // scalars: r.z alternates between out[8] and out[10] (the current one
    // and the next), out[11] = max |r|; p.q and the new r.z are summed
    // inside the update kernels from the block sums that k_zop and the last
    // sweep of the preconditioner leave in zpart
    zprecondition(P, cr, cz, s);
    BCHAR_HIP(hipMemcpyAsync(cp, cz, sizeof(double) * n2, hipMemcpyDeviceToDevice, s));
    red.dot(cr, cz, n2, 8);
    double* rz = red.out + 8;
    double* rz_next = red.out + 10;
    // iteration 0's update, then units of (preconditioner, direction,
    // product, update) advancing one iteration each; after the update of
    // iteration k the residual is checked when k % 4 == 3 or at the cap
    cg_update_half(rz, s);
    int k = 0;
    bool checked = false;   // a replayed graph has just checked iteration k
    for (;;) {
      if (!checked && ((k % 4) == 3 || k + 1 == max_cg)) {
        red.maxabs(cr, n2, 11);
        if (red.fetch(11) <= cg_tol || k + 1 == max_cg) {
          ++k;
          break;
        }
      }
      // the next check falls on iteration k + 3 (from 0) or k + 4: replay
      // those units from the graph when they all fit under the cap
      const int next = (k == 0) ? 3 : 4;
      if (graphs_ok && (k % 4) == ((k == 0) ? 0 : 3) && k + next < max_cg) {
        const int which = (k == 0) ? 0 : 1;
        // graph 0 starts from r.z in out[8], graph 1 from out[10]
        BCHAR_REQUIRE(rz == red.out + (which ? 10 : 8), BCHAR_E_DEVICE, "cg graph parity");
        if (prof_unit_due()) {
          ProfModeGuard g_(ProfMode::all);
          cg_units(next, rz, rz_next, true, s);
        } else {
          if (!G.x[which]) capture_units(which, next, rz, rz_next);
          BCHAR_HIP(hipGraphLaunch(G.x[which], s));
        }
        if (next % 2) std::swap(rz, rz_next);
        k += next;
        if (red.fetch(11) <= cg_tol || k + 1 == max_cg) {
          ++k;
          break;
        }
        checked = true;
        continue;
      }
      checked = false;
      cg_units(1, rz, rz_next, false, s);
      std::swap(rz, rz_next);
      ++k;
    }
    res.cg += k;
    red.sum(cx, n, 13);
    {
      ::bchar::ProfScope ps_("k_zdual_dir", s);
      k_zdual_dir<<<gn, kT, 0, s>>>(Q.rptr, Q.col, Q.a, cx, red.out + 13, inv_mean, n,
                                    dmu, dnu, Q.dt);
    }
    BCHAR_HIP(hipGetLastError());
    return k;
  };

  // ---------------------------------------------------------------- semismooth Newton
  // From the current t (and the per-cell multipliers in zdual that produce
  // it): Newton steps on the dual function with the generalised Jacobian
  // (entries on the box weigh 0) and a line search on its directional
  // derivative.  Returns true once max |F| <= tol; fn holds the last
  // residual.
  double fn = 0.0;
  int ssn_steps = 0;   // steps taken by semismooth Newton so far
  auto ssn = [&](double lo, double hi, int max_it, int patience, int max_cg,
                 const char* tag) -> bool {
    int short_steps = 0;
    for (int it = 0; it < max_it; ++it) {
      {
        ::bchar::ProfScope ps_("k_residual", s);
        k_residual<<<gn, kT, 0, s>>>(Q.rptr, Q.cptr, Q.cpos, Q.a, Q.ac, Q.t, nullptr, 0.0, lo, hi,
                                     Q.rr, Q.ss, n, Q.F);
      }
      zero_ghost(Q.F);
      red.maxabs(Q.F, n2, 0);
      fn = red.fetch(0);
      if (!(fn == fn)) return false;
      if (fn <= tol) return true;
      ++res.newton;
      {
        ::bchar::ProfScope ps_("k_fine_weights", s);
        // kink band: ten times the residual, at most 1e-2
        k_fine_weights<<<gz, kT, 0, s>>>(Q.a, csc.pos, Q.t, lo, hi, std::min(1e-2, 10.0 * fn),
                                         nnz, L0.w);
      }
      refresh();
      // inexact Newton: relative inner tolerance on the y-space residual,
      // near-exact once many steps were needed
      const double eta = it < 30 ? std::min(0.1, std::sqrt(fn)) * 0.1 : 1e-6;
      const double cg_tol = std::max(eta * fn, 0.1 * tol);
      const int k = pcg(Q.F, cg_tol, false, max_cg);
      if (k >= max_cg && patience > 0) {
        // a capped attempt whose linear system CG cannot solve is hopeless
        if (trace_enabled()) fprintf(stderr, "[bchar]   stop: CG did not converge\n");
        return false;
      }
      if (trace_enabled()) {
        red.maxabs(cr, n2, 11);
        fprintf(stderr, "[bchar]   newton %d%s: |F| %.3e, cg %d (|r| %.3e of %.3e), t %.3f s\n",
                it, tag, fn, k, red.fetch(11), cg_tol, wall_seconds());
      }
      // line search on phi(step) = theta(y + step d), convex and piecewise
      // quadratic: phi'(0) = F . d < 0 and phi' is nondecreasing, so any
      // step with phi'(step) <= 0 decreases theta.  The full step is taken
      // when phi'(1) <= 0; otherwise the minimiser along d is bracketed by
      // quartering and located by regula falsi (Illinois) on phi', which is
      // piecewise linear.  Directions along which the entries on the box
      // leave theta without curvature are long, and the minimiser can lie
      // many orders of magnitude below 1.
      auto dphi = [&](double al) {
        {
          ::bchar::ProfScope ps_("k_dphi_part", s);
          k_dphi_part<<<kRedBlocks, kT, 0, s>>>(Q.rptr, Q.cptr, Q.cpos, Q.a, Q.ac, Q.t, Q.dt, al,
                                                lo, hi, Q.rr, Q.ss, dmu, dnu, n, red.part);
        }
        {
          ::bchar::ProfScope ps_("k_reduce_final_sum", s);
          k_reduce_final_sum<<<1, kFinalThreads, 0, s>>>(red.part, kRedBlocks, red.out + 4);
        }
        BCHAR_HIP(hipGetLastError());
        return red.fetch(4);
      };
      const double slope = dphi(0.0);
      if (!(slope < 0.0)) {
        if (trace_enabled()) fprintf(stderr, "[bchar]   stop: slope %.3e\n", slope);
        return false;
      }
      double step = 1.0;
      const double g1 = dphi(1.0);
      int evals = 2;
      bool full = g1 <= 0.0;
      if (!full && fn < 1e-6) {
        // near the solution phi'(1) is of the order of its rounding; take a
        // full step that halves the residual
        {
          ::bchar::ProfScope ps_("k_residual", s);
          k_residual<<<gn, kT, 0, s>>>(Q.rptr, Q.cptr, Q.cpos, Q.a, Q.ac, Q.t, Q.dt, 1.0, lo, hi,
                                       Q.rr, Q.ss, n, cq);
        }
        zero_ghost(cq);
        red.maxabs(cq, n2, 14);
        full = red.fetch(14) < 0.5 * fn;
      }
      if (!full) {
        double a_lo = 0.0, g_lo = slope, a_hi = 1.0, g_hi = g1;
        for (double al = 0.25; al >= 1e-40; al *= 0.25) {
          const double g = dphi(al);
          ++evals;
          if (g <= 0.0) {
            a_lo = al;
            g_lo = g;
            break;
          }
          a_hi = al;
          g_hi = g;
        }
        if (a_lo == 0.0) {
          if (trace_enabled()) fprintf(stderr, "[bchar]   stop: no decrease along d\n");
          return false;
        }
        int side = 0;
        for (int r = 0; r < 12 && g_lo < 0.1 * slope; ++r) {
          double mid = a_lo + (a_hi - a_lo) * (g_lo / (g_lo - g_hi));
          if (!(mid > a_lo && mid < a_hi)) break;
          const double g = dphi(mid);
          ++evals;
          if (g <= 0.0) {
            a_lo = mid;
            g_lo = g;
            if (side == -1) g_hi *= 0.5;
            side = -1;
          } else {
            a_hi = mid;
            g_hi = g;
            if (side == 1) g_lo *= 0.5;
            side = 1;
          }
        }
        step = a_lo;
      }
      if (trace_enabled())
        fprintf(stderr, "[bchar]   step %.3e (%d evaluations) slope %.3e\n", step, evals, slope);
      // steps far below 1 mean directions dominated by multipliers that the
      // entries on the box leave without curvature: give up after
      // `patience` of them (0: never)
      if (step < 1e-3 && patience > 0 && ++short_steps >= patience) {
        if (trace_enabled()) fprintf(stderr, "[bchar]   stop: short steps\n");
        return false;
      }
      {
        ::bchar::ProfScope ps_("k_axpy2", s);
        k_axpy2<<<gz, kT, 0, s>>>(Q.t, Q.dt, step, nnz);
        ++ssn_steps;
      }
      {
        ::bchar::ProfScope ps_("k_zdual_acc", s);
        k_zdual_acc<<<gn, kT, 0, s>>>(cx, red.out + 13, inv_mean, step, n, zdual);
      }
      BCHAR_HIP(hipGetLastError());
      red.maxabs(Q.t, nnz, 15);
      if (!(red.fetch(15) <= 1e12)) {
        if (trace_enabled()) fprintf(stderr, "[bchar]   stop: |t| %.3e\n", red.fetch(15));
        return false;
      }
    }
    return false;
  };

  // ---------------------------------------------------------------- interior point
  // From x = 0, zl = zu = 1, t = 0, or (warm) from the current t.  Returns 2 once max |B x - r| <= tol
  // and the mean complementarity is at most kIpmMuTight (its x is then an
  // answer in its own right, within about mu / z of the minimiser), 1 when
  // it stalls after reaching 1e-10 on both, 0 when the complementarity
  // grows by 1e8 (the box admits no solution), on a NaN, or after
  // kIpmMaxIter iterations otherwise.  t and zdual are left for the
  // semismooth iteration to finish from.
  IpmArrays I{};
  I.x = ws.get<double>(nnz + 1);
  I.sl = ws.get<double>(nnz + 1);
  I.su = ws.get<double>(nnz + 1);
  I.zl = ws.get<double>(nnz + 1);
  I.zu = ws.get<double>(nnz + 1);
  I.D = ws.get<double>(nnz + 1);
  I.h = ws.get<double>(nnz + 1);
  I.dxa = ws.get<double>(nnz + 1);
  I.dx = ws.get<double>(nnz + 1);
  I.dzl = ws.get<double>(nnz + 1);
  I.dzu = ws.get<double>(nnz + 1);
  double* rp = ws.get<double>(n2);
  double fp_ipm = HUGE_VAL;
  bool ipm_diverged = false;   // the last interior point stopped with its complementarity
                               // grown by kIpmDiverged (the box looks empty)
  auto ipm = [&](double lo, double hi, bool warm, double cg_rel) -> int {
    I.lo = lo;
    I.hi = hi;
    ipm_diverged = false;
    I.has_hi = std::isinf(hi) ? 0 : 1;
    const double m_pairs = (double)nnz * (I.has_hi ? 2.0 : 1.0);
    if (warm) {
      // from the current t and zdual
      ::bchar::ProfScope ps_("k_ipm_init_warm", s);
      k_ipm_init_warm<<<gz, kT, 0, s>>>(I, Q.t, kIpmWarmShift, nnz);
    } else {
      {
        ::bchar::ProfScope ps_("k_ipm_init", s);
        k_ipm_init<<<gz, kT, 0, s>>>(I, nnz);
      }
      fill_f64(Q.t, 0.0, nnz, s);
      fill_f64(zdual, 0.0, 2 * n2, s);
    }
    BCHAR_HIP(hipGetLastError());
    double mu0 = -1.0, fp_best = HUGE_VAL;
    std::vector<double> fp_hist, mu_hist;
    const bool loose = cg_rel > kIpmCgTight;
    int stall = 0, stall_near = 0;
    auto steps = [&](double* ap, double* ad) {
      {
        ::bchar::ProfScope ps_("k_reduce_final_max", s);
        k_reduce_final_max<<<1, 64, 0, s>>>(red.part, kRedBlocks, red.out + 2);
        k_reduce_final_max<<<1, 64, 0, s>>>(red.part + kRedBlocks, kRedBlocks, red.out + 3);
      }
      double v[2];
      BCHAR_HIP(hipMemcpyAsync(v, red.out + 2, sizeof(v), hipMemcpyDeviceToHost, s));
      BCHAR_HIP(hipStreamSynchronize(s));
      *ap = v[0] > 0.0 ? 1.0 / v[0] : HUGE_VAL;
      *ad = v[1] > 0.0 ? 1.0 / v[1] : HUGE_VAL;
    };
    for (int it = 0; it < kIpmMaxIter; ++it) {
      ++res.ipm;
      {
        ::bchar::ProfScope ps_("k_ipm_prep", s);
        k_ipm_prep<<<kRedBlocks, kT, 0, s>>>(I, nnz, red.part);
      }
      {
        ::bchar::ProfScope ps_("k_reduce_final_sum", s);
        k_reduce_final_sum<<<1, kFinalThreads, 0, s>>>(red.part, kRedBlocks, red.out + 0);
      }
      {
        ::bchar::ProfScope ps_("k_ipm_h", s);
        k_ipm_h<<<gz, kT, 0, s>>>(I, Q.t, 0, 0.0, nnz);
      }
      {
        ::bchar::ProfScope ps_("k_ipm_rhs", s);
        k_ipm_rhs<<<gn, kT, 0, s>>>(Q.rptr, Q.cptr, Q.cpos, Q.a, Q.ac, I, Q.rr, Q.ss, n, rp, Q.F);
      }
      zero_ghost(rp);
      zero_ghost(Q.F);
      BCHAR_HIP(hipGetLastError());
      red.maxabs(rp, n2, 1);
      red.maxabs(Q.F, n2, 5);
      double v[6];
      BCHAR_HIP(hipMemcpyAsync(v, red.out, sizeof(v), hipMemcpyDeviceToHost, s));
      BCHAR_HIP(hipStreamSynchronize(s));
      const double mu = v[0] / m_pairs, fp = v[1], fv = v[5];
      if (mu0 < 0.0) mu0 = mu;
      fn = fp;
      if (trace_enabled())
        fprintf(stderr, "[bchar]   ipm %d: |B x - r| %.3e, mu %.3e, cg %d, t %.3f s\n", it, fp,
                mu, res.cg, wall_seconds());
      if (!(mu == mu) || !(fp == fp) || mu > 1e8 * mu0) return 0;
      // no progress on an infeasible box: after kIpmInfeasIt iterations the
      // complementarity is not below half its start and has not halved
      // over the last five either, and |B x - r| fell by less than 10 %
      // over them (a feasible box whose answer lies far from the start can
      // first drive the complementarity up by orders of magnitude, then
      // bring it down)
      fp_hist.push_back(fp);
      mu_hist.push_back(mu);
      if (it >= kIpmInfeasIt && mu >= 0.5 * mu0 && mu >= 0.5 * mu_hist[it - 5] &&
          fp >= 0.9 * fp_hist[it - 5]) {
        if (trace_enabled()) fprintf(stderr, "[bchar]   stop: no progress (infeasible?)\n");
        ipm_diverged = mu >= kIpmDiverged * mu0;
        return 0;
      }
      // loose directions that no longer reduce |B x - r| (by 10 % over
      // three iterations) hand over to a run with near-exact ones
      if (loose && it >= 3 && fp >= 0.9 * fp_hist[it - 3]) {
        if (trace_enabled()) fprintf(stderr, "[bchar]   stop: loose directions stall\n");
        return 0;
      }
      fp_ipm = fp;
      if (fp <= tol && mu <= kIpmMuTight) return 2;
      if (fp_best <= 1e-10 && mu <= 1e-10 && fp > 0.5 * fp_best) {
        // stalled: |B x - r| no longer halves
        if (++stall >= 2) return 1;
      } else if (fp_best <= kIpmNearFeasible && mu <= kIpmMuFloor && fp > 0.5 * fp_best) {
        // the complementarity is at rounding level and |B x - r| creeps:
        // the directions are as exact as CG makes them on these systems
        if (++stall_near >= 4) return 1;
      }
      if (fp < fp_best) fp_best = fp;
      {
        ::bchar::ProfScope ps_("k_ipm_weights", s);
        k_ipm_weights<<<gz, kT, 0, s>>>(Q.a, csc.pos, I.D, nnz, L0.w);
      }
      refresh();
      // inexact directions: the CG residual of the normal equations is kept
      // below cg_rel times both the right-hand side and the complementarity
      // mu, the scale at which the iterate itself is still inexact (the step
      // is re-measured at the next iterate, and the exit test above is exact)
      const double cg_tol = std::max(cg_rel * std::min(fv, mu), 1e-15);
      // predictor (affine scaling).  Once the normal equations are too
      // ill-conditioned for CG to reach its tolerance the step would spoil
      // the iterate: hand it over as it is.
      if (pcg(Q.F, cg_tol, false, o.qp_max_cg) >= o.qp_max_cg) {
        if (fp_best <= 1e-10) return 1;
        if (loose) return 0;   // too ill-conditioned for loose directions
      }
      {
        ::bchar::ProfScope ps_("k_ipm_dir", s);
        k_ipm_dir<<<kRedBlocks, kT, 0, s>>>(I, Q.dt, 0, 0.0, nnz, red.part);
      }
      double ap, ad;
      steps(&ap, &ad);
      ap = std::min(1.0, ap);
      ad = std::min(1.0, ad);
      {
        ::bchar::ProfScope ps_("k_ipm_muaff", s);
        k_ipm_muaff<<<kRedBlocks, kT, 0, s>>>(I, ap, ad, nnz, red.part);
      }
      {
        ::bchar::ProfScope ps_("k_reduce_final_sum", s);
        k_reduce_final_sum<<<1, kFinalThreads, 0, s>>>(red.part, kRedBlocks, red.out + 4);
      }
      const double mua = red.fetch(4) / m_pairs;
      const double sig = std::pow(std::max(mua, 0.0) / mu, 3.0);
      const double smu = sig * mu;
      // corrector (centring and second-order terms)
      {
        ::bchar::ProfScope ps_("k_ipm_h", s);
        k_ipm_h<<<gz, kT, 0, s>>>(I, Q.t, 1, smu, nnz);
      }
      {
        ::bchar::ProfScope ps_("k_ipm_rhs", s);
        k_ipm_rhs<<<gn, kT, 0, s>>>(Q.rptr, Q.cptr, Q.cpos, Q.a, Q.ac, I, Q.rr, Q.ss, n, rp, Q.F);
      }
      zero_ghost(rp);
      zero_ghost(Q.F);
      // the corrector's system differs from the predictor's in the
      // right-hand side only: start CG from the predictor's solution
      if (pcg(Q.F, cg_tol, true, o.qp_max_cg) >= o.qp_max_cg) {
        if (fp_best <= 1e-10) return 1;
        if (loose) return 0;
      }
      {
        ::bchar::ProfScope ps_("k_ipm_dir", s);
        k_ipm_dir<<<kRedBlocks, kT, 0, s>>>(I, Q.dt, 1, smu, nnz, red.part);
      }
      steps(&ap, &ad);
      ap = std::min(1.0, 0.995 * ap);
      ad = std::min(1.0, 0.995 * ad);
      {
        ::bchar::ProfScope ps_("k_ipm_update", s);
        k_ipm_update<<<gz, kT, 0, s>>>(I, Q.t, Q.dt, ap, ad, nnz);
      }
      {
        ::bchar::ProfScope ps_("k_zdual_acc", s);
        k_zdual_acc<<<gn, kT, 0, s>>>(cx, red.out + 13, inv_mean, ad, n, zdual);
      }
      BCHAR_HIP(hipGetLastError());
    }
    return fp_best <= 1e-10 ? 1 : 0;
  };

  // ---------------------------------------------------------------- crossover
  // From an interior point at the tolerance: keep its split of the entries
  // into those on a bound and the free ones, and solve the constraints for
  // the multipliers with that split (linear in them: a Newton step is
  // exact up to CG); accepted only if clip(t) then meets the tolerance, so
  // that x = clip(t) is the exact minimiser.  If it does not, the split is
  // read again off the new multipliers (t below / above the box: pinned,
  // else free) and the solve repeated: a primal-dual active-set iteration
  // from a start that is nearly right.  The caller restores the state when
  // every round fails.
  int8_t* side = ws.get<int8_t>((size_t)nnz + 1);
  auto crossover = [&](double lo, double hi) -> bool {
    {
      ::bchar::ProfScope ps_("k_xover_state", s);
      k_xover_state<<<gz, kT, 0, s>>>(I, kCrossoverRatio, nnz, side);
    }
    BCHAR_HIP(hipGetLastError());
    // round 0: the interior point's sides, kCrossoverSteps steps; each
    // later round: the sides read off t, one step, and no further round
    // unless the residual fell tenfold (the split is not settling)
    double f_prev = HUGE_VAL;
    int round = 0, left = kCrossoverSteps;
    for (int it = 0; round <= kCrossoverRounds; ++it) {
      if (left == 0) {
        ++round;
        left = 1;
        if (round > kCrossoverRounds) break;
        {
          ::bchar::ProfScope ps_("k_side_from_t", s);
          k_side_from_t<<<gz, kT, 0, s>>>(Q.t, lo, hi, nnz, side);
        }
        BCHAR_HIP(hipGetLastError());
      }
      --left;
      {
        ::bchar::ProfScope ps_("k_residual_sides", s);
        k_residual_sides<<<gn, kT, 0, s>>>(Q.rptr, Q.cptr, Q.cpos, Q.a, Q.ac, Q.t, side, lo, hi,
                                           Q.rr, Q.ss, n, Q.F);
      }
      zero_ghost(Q.F);
      {
        ::bchar::ProfScope ps_("k_side_weights", s);
        k_side_weights<<<gz, kT, 0, s>>>(Q.a, csc.pos, side, nnz, L0.w);
      }
      refresh();
      pcg(Q.F, 0.1 * tol, false, o.qp_max_cg);
      {
        ::bchar::ProfScope ps_("k_axpy2", s);
        k_axpy2<<<gz, kT, 0, s>>>(Q.t, Q.dt, 1.0, nnz);
      }
      {
        ::bchar::ProfScope ps_("k_zdual_acc", s);
        k_zdual_acc<<<gn, kT, 0, s>>>(cx, red.out + 13, inv_mean, 1.0, n, zdual);
      }
      {
        ::bchar::ProfScope ps_("k_residual", s);
        k_residual<<<gn, kT, 0, s>>>(Q.rptr, Q.cptr, Q.cpos, Q.a, Q.ac, Q.t, nullptr, 0.0, lo, hi,
                                     Q.rr, Q.ss, n, Q.F);
      }
      zero_ghost(Q.F);
      red.maxabs(Q.F, n2, 0);
      const double f = red.fetch(0);
      if (trace_enabled())
        fprintf(stderr, "[bchar]   crossover %d: |F| of clip(t) %.3e, cg %d, t %.3f s\n", it, f,
                res.cg, wall_seconds());
      if (f <= tol) {
        fn = f;
        return true;
      }
      if (left == 0) {
        if (round > 0 && !(f < 0.1 * f_prev)) break;
        f_prev = f;
      }
    }
    return false;
  };

  // ---------------------------------------------------------------- equality correction
  // An interior point that stalls near the tolerance on a box level (the
  // directions no longer improve |B x - r|, and semismooth Newton from its
  // t does not converge either) has an x in the box that meets the
  // constraints to about 1e-10.  The least-norm correction d with
  // B d = r - B x (Newton steps of the equality-only problem, all weights
  // a_k^2, repeated while they reduce the residual: the relative shift of
  // the Newton matrix lets each remove only part of it) puts it on the
  // constraints, so that mass is conserved to rounding.  Weighting the
  // correction by the interior point's own scaling (moving only the entries
  // away from the box) gives systems that CG does not solve here.  So an
  // entry on the box may leave it by its share of d: a sliver a_k can take
  // a share far above |d| relative to a_k, while its volume a_k (1 + x_k)
  // moves by a_k d_k, of the order of the residual removed.  The
  // multipliers are the interior point's (zsave).
  auto equality_correction = [&]() -> bool {
    BCHAR_HIP(hipMemcpyAsync(Q.t, I.x, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
    BCHAR_HIP(hipMemcpyAsync(zdual, zsave, sizeof(double) * 2 * n2, hipMemcpyDeviceToDevice, s));
    {
      ::bchar::ProfScope ps_("k_fine_weights", s);
      k_fine_weights<<<gz, kT, 0, s>>>(Q.a, csc.pos, Q.t, -HUGE_VAL, HUGE_VAL, 0.0, nnz, L0.w);
    }
    BCHAR_HIP(hipGetLastError());
    refresh();
    double f_prev = HUGE_VAL;
    for (int it = 0; it < kCorrectionSteps; ++it) {
      {
        ::bchar::ProfScope ps_("k_residual", s);
        k_residual<<<gn, kT, 0, s>>>(Q.rptr, Q.cptr, Q.cpos, Q.a, Q.ac, Q.t, nullptr, 0.0,
                                     -HUGE_VAL, HUGE_VAL, Q.rr, Q.ss, n, Q.F);
      }
      zero_ghost(Q.F);
      red.maxabs(Q.F, n2, 0);
      fn = red.fetch(0);
      if (trace_enabled())
        fprintf(stderr, "[bchar]   equality correction %d: |B x - r| %.3e, cg %d\n", it, fn,
                res.cg);
      if (!(fn == fn)) return false;
      if (fn <= tol) return true;
      if (!(fn < 0.9 * f_prev)) return false;
      f_prev = fn;
      pcg(Q.F, 0.1 * tol, false, o.qp_max_cg);
      {
        ::bchar::ProfScope ps_("k_axpy2", s);
        k_axpy2<<<gz, kT, 0, s>>>(Q.t, Q.dt, 1.0, nnz);
      }
      BCHAR_HIP(hipGetLastError());
    }
    return false;
  };

  // ---------------------------------------------------------------- box levels
  // Level 0 is the paper's box, level 1 keeps x >= -1 only, level 2 keeps
  // the equalities alone.  A level with a bound is solved by the interior
  // point followed by semismooth Newton (kPolishNewton steps at most), or,
  // when the previous solve of this transfer ended at the same level, by
  // semismooth Newton from its multipliers first (kWarmNewton steps of at
  // most kPolishCG CG iterations each).  The answer is clip(t) when semismooth Newton reaches the
  // tolerance, else the interior point's x if it reached it.  An interior
  // point that fails declares the level infeasible.
  const double lo_levels[3] = {-1.0, -1.0, -HUGE_VAL};
  const double hi_levels[3] = {1.0, HUGE_VAL, HUGE_VAL};
  // the caller may stop at level 1 (it halves the step rather than accept
  // negative volumes)
  const int max_level = o.box_policy == BCHAR_BOX_STRICT ? 0 : (o.halve_on_level2 ? 1 : 2);
  bool converged = false, ipm_answer = false, corrected = false;
  // The answer of a level from an interior point that ended at (r = 2) or
  // near (r = 1) the tolerance: crossover, semismooth polish, its own x,
  // or the equality correction (sets converged, ipm_answer, corrected).
  auto finish_interior_point = [&](int r, double lo, double hi) {
    // an interior point at the tolerance is an answer already: one
    // short semismooth step is enough to give up on the exact one.  Its
    // multipliers and t are kept, so that an interior-point answer leaves
    // the multipliers that go with its x (and the next solve's warm
    // start) rather than those of an abandoned step.
    BCHAR_HIP(hipMemcpyAsync(zsave, zdual, sizeof(double) * 2 * n2, hipMemcpyDeviceToDevice, s));
    BCHAR_HIP(hipMemcpyAsync(tsave, Q.t, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
    if (r == 2) {
      converged = crossover(lo, hi);
      if (!converged) {
        BCHAR_HIP(hipMemcpyAsync(zdual, zsave, sizeof(double) * 2 * n2, hipMemcpyDeviceToDevice,
                                 s));
        BCHAR_HIP(hipMemcpyAsync(Q.t, tsave, sizeof(double) * nnz, hipMemcpyDeviceToDevice,
                                 s));
      }
    }
    if (!converged)
      converged = ssn(lo, hi, std::min(kPolishNewton, o.qp_max_newton), r == 2 ? 1 : 2,
                      r == 2 ? std::min(kPolishCG, o.qp_max_cg) : o.qp_max_cg,
                      " (after interior point)");
    if (!converged && r == 2) {
      converged = ipm_answer = true;
      fn = fp_ipm;
      BCHAR_HIP(hipMemcpyAsync(zdual, zsave, sizeof(double) * 2 * n2, hipMemcpyDeviceToDevice, s));
      BCHAR_HIP(hipMemcpyAsync(Q.t, tsave, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
    } else if (!converged) {
      // the interior point stalled short of the tolerance: semismooth
      // Newton without the step-count cap, as long as its steps are not
      // all short, then the equality correction of the interior
      // point's x
      converged = ssn(lo, hi, o.qp_max_newton, kFallbackPatience, o.qp_max_cg,
                      " (after interior point)");
      if (!converged) converged = corrected = equality_correction();
    }
  };
  int level = 0;
  for (level = 0; level <= max_level; ++level) {
    const double lo = lo_levels[level], hi = hi_levels[level];
    if (o.warm_start && warm_level == level) {
      {
        ::bchar::ProfScope ps_("k_t_from_z", s);
        k_t_from_z<<<gn, kT, 0, s>>>(Q.rptr, Q.col, Q.a, zdual, n, Q.t);
      }
      BCHAR_HIP(hipGetLastError());
      // t is formed from the leading parts: the compensation starts anew
      fill_f64(zdual + n2, 0.0, n2, s);
      // a warm attempt that failed before its first step (its first
      // system beyond kPolishCG iterations) is not repeated on the next
      // few solves (the flow keeps changing as much from step to step):
      // they go to the warm interior point at once.  An attempt that took
      // steps leaves the interior point a better start and is kept.
      if (warm_newton_skip > 0) {
        --warm_newton_skip;
      } else {
        const int steps_before = ssn_steps;
        converged = ssn(lo, hi, std::min(kWarmNewton, o.qp_max_newton), 2,
                        std::min(kPolishCG, o.qp_max_cg), " (warm)");
        if (!converged && ssn_steps == steps_before) warm_newton_skip = kWarmNewtonPause;
      }
      if (converged) break;
    }
    const bool warm = o.warm_start && warm_level == level;
    if (level == 2) {
      fill_f64(Q.t, 0.0, nnz, s);
      fill_f64(zdual, 0.0, 2 * n2, s);
      converged = ssn(lo, hi, o.qp_max_newton, 0, o.qp_max_cg, "");
    } else {
      // a warm or loose interior point that fails is retried from zero,
      // then with near-exact directions
      int r = warm ? ipm(lo, hi, true, kIpmCgLoose) : 0;
      if (r == 0) r = ipm(lo, hi, false, kIpmCgLoose);
      if (r == 0) r = ipm(lo, hi, false, kIpmCgTight);
      if (r > 0) {
        finish_interior_point(r, lo, hi);
      } else if (level == 1) {
        // every interior point from x = 0 gave up on the box x >= -1: an
        // answer far from that start (some x of order 1 or more) can stall
        // it as if the box were empty.  One more interior point starts
        // from the minimiser of the equalities alone (a linear problem:
        // semismooth Newton without a box, a few steps), whose entries
        // below -1 it moves into the box; then semismooth Newton from zero
        // decides before the equalities alone (which allow negative
        // volumes) are taken: on an empty box both stall.  (The paper's
        // box, level 0, is empty often enough that the interior point's
        // conclusion stands.)
        fill_f64(Q.t, 0.0, nnz, s);
        fill_f64(zdual, 0.0, 2 * n2, s);
        // (not when the last one's complementarity blew up: the box then
        // looks empty, and the restart would only confirm it)
        if (!ipm_diverged &&
            ssn(-HUGE_VAL, HUGE_VAL, std::min(kFallbackNewton, o.qp_max_newton), kFallbackPatience,
                o.qp_max_cg, " (equalities alone, start of an interior point)")) {
          const int r2 = ipm(lo, hi, true, kIpmCgTight);
          if (r2 > 0) finish_interior_point(r2, lo, hi);
        }
        if (!converged) {
          fill_f64(Q.t, 0.0, nnz, s);
          fill_f64(zdual, 0.0, 2 * n2, s);
          // patient: from zero the answer may take dozens of short steps
          // (the non-solenoidal swirl at 32^3 needs about 40); a Newton
          // system that CG cannot solve still ends it at once
          converged = ssn(lo, hi, std::min(kFallbackNewtonLong, o.qp_max_newton),
                          kFallbackPatienceLong, o.qp_max_cg, " (interior point failed)");
        }
      }
    }
    if (converged) break;
  }
  res.residual = fn;
  if (!converged) {
    res.level = level > max_level ? max_level : level;
    return max_level < 2 ? BCHAR_E_QP_INFEASIBLE : BCHAR_E_QP_NOT_CONVERGED;
  }
  res.level = level;
  {
    ::bchar::ProfScope ps_("k_mu_nu", s);
    k_mu_nu<<<gn, kT, 0, s>>>(zdual, n, mu_out, nu_out);
  }
  const double lo = lo_levels[level], hi = hi_levels[level];
  int32_t* counts = ws.get<int32_t>(2);
  fill_i32(counts, 0, 2, s);
  {
    ::bchar::ProfScope ps_("k_final", s);
    // a corrected x is taken as it is (it may leave the box by its share of
    // the correction); entries within 1e-12 of a bound, or beyond it, count
    // as on it
    if (corrected)
      k_final<<<gz, kT, 0, s>>>(AN, Q.t, nullptr, lo, hi, 1e-12, 0, nnz, x_out, A_out, counts);
    else
      k_final<<<gz, kT, 0, s>>>(AN, Q.t, ipm_answer ? I.x : nullptr, lo, hi,
                                ipm_answer ? 1e-12 : 0.0, 1, nnz, x_out, A_out, counts);
  }
  BCHAR_HIP(hipGetLastError());
  int32_t hc[2];
  BCHAR_HIP(hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, s));
  BCHAR_HIP(hipStreamSynchronize(s));
  res.corrected = corrected;
  res.at_lower = hc[0];
  res.at_upper = hc[1];
  return BCHAR_OK;
}

}  // namespace bchar
