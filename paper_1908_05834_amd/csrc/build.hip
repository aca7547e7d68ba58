// Tracking (Sec. 2, eq. charac) and the initial approximation V
// (Sec. 3.1, eqs. fracMaterial and ball_int) assembled as CSR.
//
// trace:   one thread per ball, classical RK4 backward over dt with the
//          velocity frozen (multilinear lattice interpolation), v = u/phi,
//          result clamped into the domain box.  With non-constant phi the
//          2d points C +- r e_a are tracked too and r_hat is the mean of
//          their distances to the tracked centre (eq. rTrackedBall); phi(x)
//          is that of the Cartesian cell floor((x - o) / h), or, on a
//          simplicial mesh, of the cell located through a uniform grid of
//          cell lists (the rule is stated in bchar.h).
// assemble: one pass.  A workgroup of 256 threads takes a tile of cells
//          (a block of 4x4x2 / 8x8 cells on a Cartesian mesh, a run of
//          consecutive cells otherwise) and one thread per tracked ball of
//          those cells.  Each thread walks the rows of hash buckets around
//          its tracked centre (a row of buckets is one contiguous run of
//          bucket slots) and, for every overlapping residing ball
//          (predicate without sqrt or FMA, tangency excluded), forms the
//          weight omega = rho_M phi_M |B_hat cap B| and S = sum omega; a
//          block scan places every ball's overlaps, a second walk (from
//          cache) writes the shares rho_K phi_K |B| omega / S into LDS, and
//          the threads of each cell merge them by residing cell M (sorted,
//          summed in a fixed order).  A tile whose overlaps exceed the LDS
//          capacity is processed in groups of whole cells.  Each group
//          reserves room in a staging array with one atomic add; a scan of
//          the row lengths and a copy kernel then lay the rows out as CSR.
//          No floating-point atomics: the values do not depend on
//          scheduling (only the staging positions do).
#include <cmath>
#include <type_traits>

#include "device_util.hpp"
#include "internal.hpp"

namespace bchar {

// ---------------------------------------------------------------- tracking

template <class T>
struct VelocityView {
  const T* u[3];
  int64_t m[3];
  T org[3], sp[3], upper[3];
};

template <class T>
struct PhiView {
  const double* phi;   // per cell (binary64)
  bool constant;
  T phi0;
  int64_t n[3];
  T org[3], h[3];
  // simplicial meshes (simplex != 0): vertices SoA, (dim+1) ids per cell,
  // centroids (SoA), the domain box and the location grid
  int simplex;
  const double* vtx;
  int64_t n_vertices;
  const int32_t* cells;
  const double* cen;
  int64_t n_cells;
  double box_lo[3], box_hi[3];
  double pl_inv;
  int64_t pl_nb[3];
  const int32_t* pl_start;
  const int32_t* pl_list;
};

// d! times the signed measure of the simplex (a, b, c[, d]): the
// determinant of the edges from a expanded along the first edge, each
// operation rounded on its own in the order written.
template <int DIM>
__device__ __forceinline__ double orient(const double* a, const double* b, const double* c,
                                         const double* d) {
#pragma clang fp contract(off)
  double e1[3], e2[3], e3[3];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    e1[k] = b[k] - a[k];
    e2[k] = c[k] - a[k];
    if (DIM == 3) e3[k] = d[k] - a[k];
  }
  if (DIM == 2) return e1[0] * e2[1] - e1[1] * e2[0];
  const double m0 = e2[1] * e3[2] - e2[2] * e3[1];
  const double m1 = e2[0] * e3[2] - e2[2] * e3[0];
  const double m2 = e2[0] * e3[1] - e2[1] * e3[0];
  return (e1[0] * m0 - e1[1] * m1) + e1[2] * m2;
}

// Cell of a simplicial mesh holding x (already inside the domain box):
// among the cells listed in x's grid cell whose bounding box holds x, the
// lowest-numbered one whose orientation tests with each vertex replaced by
// x agree in sign with its own orientation or vanish; else the one whose
// centroid is nearest (lowest number on ties).
template <int DIM, class T>
__device__ int64_t locate(const PhiView<T>& P, const double x[3]) {
#pragma clang fp contract(off)
  int64_t g = 0, stride = 1;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    int64_t i = (int64_t)floor((x[a] - P.box_lo[a]) * P.pl_inv);
    i = i < 0 ? 0 : (i >= P.pl_nb[a] ? P.pl_nb[a] - 1 : i);
    g += i * stride;
    stride *= P.pl_nb[a];
  }
  int64_t best = -1;
  double best_d2 = 0.0;
  for (int32_t e = P.pl_start[g]; e < P.pl_start[g + 1]; ++e) {
    const int32_t K = P.pl_list[e];
    double v[DIM + 1][3];
    bool in_box = true;
#pragma unroll
    for (int i = 0; i <= DIM; ++i) {
      const int32_t q = P.cells[(int64_t)K * (DIM + 1) + i];
#pragma unroll
      for (int a = 0; a < DIM; ++a) v[i][a] = P.vtx[a * P.n_vertices + q];
      if (DIM == 2) v[i][2] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      double lo = v[0][a], hi = v[0][a];
#pragma unroll
      for (int i = 1; i <= DIM; ++i) {
        lo = v[i][a] < lo ? v[i][a] : lo;
        hi = v[i][a] > hi ? v[i][a] : hi;
      }
      in_box = in_box && x[a] >= lo && x[a] <= hi;
    }
    if (!in_box) continue;
    const double own = orient<DIM>(v[0], v[1], v[2], v[DIM == 3 ? 3 : 2]);
    bool inside = own != 0.0;
#pragma unroll
    for (int i = 0; i <= DIM; ++i) {
      if (!inside) break;
      const double* w[4] = {v[0], v[1], v[2], v[DIM == 3 ? 3 : 2]};
      w[i] = x;
      const double o = orient<DIM>(w[0], w[1], w[2], w[3]);
      inside = own > 0.0 ? o >= 0.0 : o <= 0.0;
    }
    if (inside) return K;
    // fallback candidate: nearest centroid
    double d = x[0] - P.cen[K];
    double d2 = d * d;
    d = x[1] - P.cen[P.n_cells + K];
    d2 = d2 + d * d;
    if (DIM == 3) {
      d = x[2] - P.cen[2 * P.n_cells + K];
      d2 = d2 + d * d;
    }
    if (best < 0 || d2 < best_d2) {
      best = K;
      best_d2 = d2;
    }
  }
  return best < 0 ? 0 : best;
}

// Lattice cell and local coordinates of a query: the query is clamped
// into the lattice box, t = (q - origin) / spacing, the lattice cell is
// floor(t) clamped to [0, m - 2], f = t - cell.
template <int DIM, class T>
__device__ __forceinline__ void q1_cell(const VelocityView<T>& V, const T x[3], int64_t idx[3],
                                        T f[3]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    T q = x[a] < V.org[a] ? V.org[a] : (x[a] > V.upper[a] ? V.upper[a] : x[a]);
    T t = (q - V.org[a]) / V.sp[a];
    int64_t i = (int64_t)floor(t);
    if (i > V.m[a] - 2) i = V.m[a] - 2;
    if (i < 0) i = 0;
    idx[a] = i;
    f[a] = t - (T)i;
  }
}

// Multilinear interpolation, written as the sum over the 2^d lattice
// corners of (product of the per-axis weights f or 1 - f) times the nodal
// value, corners in binary order, axes in order.  Every operation is
// rounded on its own (no contraction), so that binary64 tracking is
// reproducible operation by operation.
template <int DIM, class T>
__device__ __forceinline__ void q1(const VelocityView<T>& V, const T x[3], T out[3]) {
#pragma clang fp contract(off)
  int64_t idx[3] = {0, 0, 0};
  T f[3] = {0, 0, 0};
  q1_cell<DIM, T>(V, x, idx, f);
  const int64_t stride[3] = {1, V.m[0], V.m[0] * V.m[1]};
#pragma unroll
  for (int c = 0; c < DIM; ++c) out[c] = 0;
#pragma unroll
  for (int corner = 0; corner < (1 << DIM); ++corner) {
    T w = 1;
    int64_t node = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const int bit = (corner >> a) & 1;
      w = w * (bit ? f[a] : (T)1 - f[a]);
      node += (idx[a] + bit) * stride[a];
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) out[c] = out[c] + w * V.u[c][node];
  }
}

// div of the Q1 interpolant at x (same lattice cell as q1): per axis a,
// the corners in binary order add (+ if the corner's bit a is set, else
// -) the product of the other axes' weights times u_a at the corner, the
// sum is divided by the spacing of a; the axes' terms are added in order.
template <int DIM, class T>
__device__ __forceinline__ T q1_div(const VelocityView<T>& V, const T x[3]) {
#pragma clang fp contract(off)
  int64_t idx[3] = {0, 0, 0};
  T f[3] = {0, 0, 0};
  q1_cell<DIM, T>(V, x, idx, f);
  const int64_t stride[3] = {1, V.m[0], V.m[0] * V.m[1]};
  T div = 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    T acc = 0;
#pragma unroll
    for (int corner = 0; corner < (1 << DIM); ++corner) {
      T g = 1;
      int64_t node = 0;
#pragma unroll
      for (int b = 0; b < DIM; ++b) {
        const int bit = (corner >> b) & 1;
        if (b != a) g = g * (bit ? f[b] : (T)1 - f[b]);
        node += (idx[b] + bit) * stride[b];
      }
      const T term = g * V.u[a][node];
      acc = ((corner >> a) & 1) ? acc + term : acc - term;
    }
    div = div + acc / V.sp[a];
  }
  return div;
}

// phi of the cell containing x (floor((x - origin) / h), clamped; on a
// simplicial mesh the located cell of x clamped into the domain box), or
// the common value when phi is constant.
template <int DIM, class T>
__device__ __forceinline__ T phi_at(const PhiView<T>& P, const T x[3]) {
#pragma clang fp contract(off)
  if (P.constant) return P.phi0;
  if (P.simplex) {
    double q[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const double xa = (double)x[a];
      q[a] = xa < P.box_lo[a] ? P.box_lo[a] : (xa > P.box_hi[a] ? P.box_hi[a] : xa);
    }
    return (T)P.phi[locate<DIM, T>(P, q)];
  }
  int64_t cid = 0, stride = 1;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    int64_t i = (int64_t)floor((x[a] - P.org[a]) / P.h[a]);
    i = i < 0 ? 0 : (i >= P.n[a] ? P.n[a] - 1 : i);
    cid += i * stride;
    stride *= P.n[a];
  }
  return (T)P.phi[cid];
}

// v = u / phi at x; with GROW also delta = div u / phi, the rate at which
// the flow of u / phi dilates volume in a cell of constant porosity.
template <int DIM, class T, bool GROW>
__device__ __forceinline__ void speed(const VelocityView<T>& V, const PhiView<T>& P,
                                      const T x[3], T v[3], T* delta) {
#pragma clang fp contract(off)
  q1<DIM, T>(V, x, v);
  const T ph = phi_at<DIM, T>(P, x);
#pragma unroll
  for (int a = 0; a < DIM; ++a) v[a] = v[a] / ph;
  if (GROW) *delta = q1_div<DIM, T>(V, x) / ph;
}

// One classical RK4 step per sub-interval, backward: stage points
// X - (tau/2) k1, X - (tau/2) k2, X - tau k3, update
// X - (tau/6) (((k1 + 2 k2) + 2 k3) + k4), then clamp into the box.
// With GROW the log growth lam of a carried region's porous volume takes
// the same stages: lam - (tau/6) (((d1 + 2 d2) + 2 d3) + d4) with d the
// dilation rate at the stage points (Liouville along the path).
template <int DIM, class T, bool GROW>
__device__ __forceinline__ void rk4_back(const VelocityView<T>& V, const PhiView<T>& P, T X[3],
                                         T tau, int substeps, const T lo[3], const T hi[3],
                                         T* lam) {
#pragma clang fp contract(off)
  const T htau = (T)0.5 * tau;
  const T tau6 = tau / (T)6;
  for (int st = 0; st < substeps; ++st) {
    T k1[3], k2[3], k3[3], k4[3], y[3];
    T d1 = 0, d2 = 0, d3 = 0, d4 = 0;
    speed<DIM, T, GROW>(V, P, X, k1, &d1);
#pragma unroll
    for (int a = 0; a < DIM; ++a) y[a] = X[a] - htau * k1[a];
    speed<DIM, T, GROW>(V, P, y, k2, &d2);
#pragma unroll
    for (int a = 0; a < DIM; ++a) y[a] = X[a] - htau * k2[a];
    speed<DIM, T, GROW>(V, P, y, k3, &d3);
#pragma unroll
    for (int a = 0; a < DIM; ++a) y[a] = X[a] - tau * k3[a];
    speed<DIM, T, GROW>(V, P, y, k4, &d4);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      T acc = k1[a] + (T)2 * k2[a];
      acc = acc + (T)2 * k3[a];
      acc = acc + k4[a];
      T xa = X[a] - tau6 * acc;
      xa = xa > lo[a] ? xa : lo[a];
      X[a] = xa < hi[a] ? xa : hi[a];
    }
    if (GROW) {
      T acc = d1 + (T)2 * d2;
      acc = acc + (T)2 * d3;
      acc = acc + d4;
      *lam = *lam - tau6 * acc;
    }
  }
}

// One thread per ball: the tracked centre (eq. charac), and r_hat: r when
// phi is constant and u solenoidal (eq. ball_volChange), else the mean
// distance of the 2d tracked cardinal points C +- r e_a to the tracked
// centre (eq. rTrackedBall).  GROW (non-solenoidal u) also writes the log
// growth lam of the ball's porous volume.  128 threads a block: the launch
// bound lets the binary64 RK4 state stay in registers (the default bound
// of 1024 threads caps a lane at 128 VGPRs and spills it to scratch).
template <int DIM, class T, bool GROW>
__global__ void __launch_bounds__(128) k_trace(VelocityView<T> V, PhiView<T> P,
                                               const double* __restrict__ cen,
                                               const double* __restrict__ rad, int64_t n_balls,
                                               T tau, int substeps, T lo0, T lo1, T lo2, T hi0,
                                               T hi1, T hi2, double* __restrict__ tracked,
                                               double* __restrict__ r_hat,
                                               double* __restrict__ lam_out) {
#pragma clang fp contract(off)
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_balls) return;
  const T lo[3] = {lo0, lo1, lo2};
  const T hi[3] = {hi0, hi1, hi2};
  T C[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) C[a] = (T)cen[a * n_balls + b];
  T X[3] = {C[0], C[1], C[2]};
  T lam = 0;
  rk4_back<DIM, T, GROW>(V, P, X, tau, substeps, lo, hi, &lam);
#pragma unroll
  for (int a = 0; a < DIM; ++a) tracked[a * n_balls + b] = (double)X[a];
  if (GROW) lam_out[b] = (double)lam;
  const T r = (T)rad[b];
  if (P.constant && !GROW) {
    r_hat[b] = (double)r;
    return;
  }
  // eq. rTrackedBall: mean distance of the tracked cardinal points C +- r e_a
  T acc = 0;
  for (int a = 0; a < DIM; ++a) {
    for (int sg = 0; sg < 2; ++sg) {
      T Y[3] = {C[0], C[1], C[2]};
      Y[a] = sg == 0 ? Y[a] + r : Y[a] - r;
      rk4_back<DIM, T, false>(V, P, Y, tau, substeps, lo, hi, nullptr);
      T d = Y[0] - X[0];
      T d2 = d * d;
      for (int c = 1; c < DIM; ++c) {
        d = Y[c] - X[c];
        d2 = d2 + d * d;
      }
      acc = acc + sqrt(d2);
    }
  }
  r_hat[b] = (double)(acc / (T)(2 * DIM));
}

__global__ void k_to_f32(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

template <int DIM, class T>
static void launch_trace(const bchar_mesh_s* m, const bchar_velocity& u, double dt,
                         int substeps, const T* const* comps, double* tracked, double* r_hat,
                         double* lam, hipStream_t s) {
  VelocityView<T> V;
  PhiView<T> P;
  for (int a = 0; a < 3; ++a) {
    V.u[a] = a < DIM ? comps[a] : nullptr;
    V.m[a] = a < DIM ? u.m[a] : 1;
    V.org[a] = (T)(a < DIM ? u.origin[a] : 0.0);
    V.sp[a] = (T)(a < DIM ? u.spacing[a] : 1.0);
    V.upper[a] = (T)(a < DIM ? u.origin[a] + (double)(u.m[a] - 1) * u.spacing[a] : 0.0);
    P.n[a] = m->n[a];
    P.org[a] = (T)m->origin[a];
    P.h[a] = (T)m->h[a];
  }
  P.phi = m->phi.as<double>();
  P.constant = m->phi_const;
  P.phi0 = (T)m->phi0;
  P.simplex = m->kind == BCHAR_MESH_SIMPLEX ? 1 : 0;
  P.vtx = m->vtx.as<double>();
  P.n_vertices = m->n_vertices;
  P.cells = m->cells.as<int32_t>();
  P.cen = m->cell_cen.as<double>();
  P.n_cells = m->n_cells;
  P.pl_inv = m->pl_inv;
  P.pl_start = m->pl_start.as<int32_t>();
  P.pl_list = m->pl_list.as<int32_t>();
  T lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    P.box_lo[a] = m->box_lo[a];
    P.box_hi[a] = m->box_hi[a];
    P.pl_nb[a] = m->pl_nb[a];
    lo[a] = (T)m->box_lo[a];
    hi[a] = (T)m->box_hi[a];
  }
  const T tau = (T)(dt / substeps);
  {
    ::bchar::ProfScope ps_("k_trace", s);
    // the growth is tracked in binary64 only
    if constexpr (std::is_same<T, double>::value) {
      if (lam) {
        k_trace<DIM, T, true><<<blocks_for(m->n_balls, 128), 128, 0, s>>>(
            V, P, m->cen.as<double>(), m->rad.as<double>(), m->n_balls, tau, substeps, lo[0],
            lo[1], lo[2], hi[0], hi[1], hi[2], tracked, r_hat, lam);
        BCHAR_HIP(hipGetLastError());
        return;
      }
    }
    k_trace<DIM, T, false><<<blocks_for(m->n_balls, 128), 128, 0, s>>>(
        V, P, m->cen.as<double>(), m->rad.as<double>(), m->n_balls, tau, substeps, lo[0], lo[1],
        lo[2], hi[0], hi[1], hi[2], tracked, r_hat, nullptr);
  }
  BCHAR_HIP(hipGetLastError());
}

void trace_balls(const bchar_mesh_s* m, const bchar_velocity& u, double dt, int substeps,
                 int precision, double* tracked, double* r_hat, double* lam, Arena& ws,
                 hipStream_t s) {
  // binary32 tracking only in FP32_VOLUME, which the caller allows only
  // where phi is constant and u solenoidal (on faces, where u/phi jumps and
  // the cardinal points start, binary32 rounding would pick the
  // neighbouring cell's phi)
  if (precision != BCHAR_FP32_VOLUME || lam) {
    const double* comps[3] = {u.u[0], u.u[1], u.u[2]};
    if (m->dim == 2)
      launch_trace<2, double>(m, u, dt, substeps, comps, tracked, r_hat, lam, s);
    else
      launch_trace<3, double>(m, u, dt, substeps, comps, tracked, r_hat, lam, s);
  } else {
    const int64_t nn = u.m[0] * u.m[1] * (m->dim == 3 ? u.m[2] : 1);
    const float* comps[3] = {nullptr, nullptr, nullptr};
    for (int a = 0; a < m->dim; ++a) {
      float* c = ws.get<float>(nn);
      {
        ::bchar::ProfScope ps_("k_to_f32", s);
        k_to_f32<<<blocks_for(nn, 256), 256, 0, s>>>(u.u[a], c, nn);
      }
      BCHAR_HIP(hipGetLastError());
      comps[a] = c;
    }
    if (m->dim == 2)
      launch_trace<2, float>(m, u, dt, substeps, comps, tracked, r_hat, nullptr, s);
    else
      launch_trace<3, float>(m, u, dt, substeps, comps, tracked, r_hat, nullptr, s);
  }
}

// ---------------------------------------------------------------- row targets
// Non-solenoidal u (Sec. 3.2, Remark on non-solenoidal fields): every
// tracked ball carries rho_K phi_K |B_{K,s}| exp(lam) (the analogue of
// eq. expPhiB) and their sum over the balls of K is T_K (eq. volTracked).
// The trace-back regions cover the domain once, so the targets of the
// tracked cells that take their material from a set of residing cells
// alone must total those cells' porous volumes: the sets are the connected
// components of the bipartite graph of V's pattern (row K -- column M per
// entry), and within each, b_row = T_K sum_{M in it} |M|_phi /
// sum_{K in it} T_K.  One component (the usual case) is the whole domain.

constexpr int kTargetBlocks = 256;
constexpr int kMaxCcRounds = 4096;

__global__ void __launch_bounds__(256) k_tracked_mass(
    int64_t n_cells, int nbpc, const int32_t* __restrict__ ball_ptr,
    const double* __restrict__ rho, const double* __restrict__ phi,
    const double* __restrict__ bvol, const double* __restrict__ lam,
    const double* __restrict__ b, double* __restrict__ T, double* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ double sh[32];
  CSum st, sb;
  for (int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; K < n_cells;
       K += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b0 = nbpc > 0 ? K * nbpc : ball_ptr[K];
    const int64_t b1 = nbpc > 0 ? b0 + nbpc : ball_ptr[K + 1];
    double t = 0.0;
    for (int64_t q = b0; q < b1; ++q) t = t + (rho[K] * phi[K] * bvol[q]) * exp(lam[q]);
    T[K] = t;
    st.add(t);
    sb.add(b[K]);
  }
  const CSum a = block_csum(st, sh);
  const CSum c = block_csum(sb, sh);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x] = a.hi;
    part[4 * blockIdx.x + 1] = a.lo;
    part[4 * blockIdx.x + 2] = c.hi;
    part[4 * blockIdx.x + 3] = c.lo;
  }
}

// out[0] = sum T, out[1] = sum b, out[2] = sum b / sum T (one block)
__global__ void __launch_bounds__(256) k_target_scale(const double* __restrict__ part, int np,
                                                      double* __restrict__ out) {
  __shared__ double sh[32];
  CSum st, sb;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    CSum x;
    x.hi = part[4 * i];
    x.lo = part[4 * i + 1];
    st.add(x);
    x.hi = part[4 * i + 2];
    x.lo = part[4 * i + 3];
    sb.add(x);
  }
  const double t = block_csum(st, sh).value();
  const double bb = block_csum(sb, sh).value();
  if (threadIdx.x == 0) {
    out[0] = t;
    out[1] = bb;
    out[2] = bb / t;
  }
}

// Connected components by hooking and pointer jumping.  lab[v] <= v
// always and points inside v's component; at the fixed point every node
// holds the smallest node of its component.
__global__ void k_cc_init(int64_t n2, int32_t* __restrict__ lab) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n2) lab[v] = (int32_t)v;
}

__global__ void k_cc_hook(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                          int64_t n, int32_t* lab, int32_t* __restrict__ changed) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= n) return;
  for (int32_t e = row_ptr[K]; e < row_ptr[K + 1]; ++e) {
    const int32_t a = __atomic_load_n(&lab[K], __ATOMIC_RELAXED);
    const int32_t b = __atomic_load_n(&lab[n + col[e]], __ATOMIC_RELAXED);
    if (a == b) continue;
    const int32_t hi = a > b ? a : b, lo = a > b ? b : a;
    if (atomicMin(&lab[hi], lo) > lo) *changed = 1;
  }
}

__global__ void k_cc_compress(int64_t n2, int32_t* lab) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n2) return;
  int32_t l = __atomic_load_n(&lab[v], __ATOMIC_RELAXED);
  for (;;) {
    const int32_t p = __atomic_load_n(&lab[l], __ATOMIC_RELAXED);
    if (p == l) break;
    l = p;
  }
  __atomic_store_n(&lab[v], l, __ATOMIC_RELAXED);
}

__global__ void k_cc_roots(int64_t n2, const int32_t* __restrict__ lab,
                           int32_t* __restrict__ count) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n2 && lab[v] == (int32_t)v) atomicAdd(count, 1);
}

// One wave per label: sum of T over the component's rows and of b over
// its columns (members in ascending node order), and their ratio.
__global__ void __launch_bounds__(64) k_cc_scale(int64_t n, const int32_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ perm,
                                                 const double* __restrict__ T,
                                                 const double* __restrict__ b,
                                                 double* __restrict__ scale) {
  const int64_t c = blockIdx.x;
  const int32_t p0 = ptr[c], p1 = ptr[c + 1];
  if (p0 == p1) return;
  CSum st, sb;
  for (int32_t q = p0 + (int32_t)threadIdx.x; q < p1; q += 64) {
    const int64_t v = perm[q];
    if (v < n)
      st.add(T[v]);
    else
      sb.add(b[v - n]);
  }
  wave_csum(st);
  wave_csum(sb);
  if (threadIdx.x == 0) scale[c] = sb.value() / st.value();
}

__global__ void k_scale_targets(int64_t n, const double* __restrict__ T,
                                const int32_t* __restrict__ lab,
                                const double* __restrict__ scale, double* __restrict__ b_row) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K < n) b_row[K] = T[K] * scale[lab ? lab[K] : 0];
}

TargetInfo row_targets(const bchar_mesh_s* m, bchar_transfer_s* t, const double* lam,
                       double* b_row, Arena& ws, hipStream_t s) {
  const int64_t n = m->n_cells, n2 = 2 * n;
  const int32_t* row_ptr = t->row_ptr.as<int32_t>();
  const int32_t* col = t->col.as<int32_t>();
  Arena::Mark mk = ws.mark();
  double* T = ws.get<double>(n);
  double* part = ws.get<double>(4 * kTargetBlocks);
  double* out = ws.get<double>(4);
  t->grp_lab.reserve(sizeof(int32_t) * n2);
  int32_t* lab = t->grp_lab.as<int32_t>();
  int32_t* flag = ws.get<int32_t>(2);
  {
    ::bchar::ProfScope ps_("k_tracked_mass", s);
    k_tracked_mass<<<kTargetBlocks, 256, 0, s>>>(
        n, m->nbpc, m->ball_ptr.as<int32_t>(), m->rho.as<double>(), m->phi.as<double>(),
        m->bvol.as<double>(), lam, m->b.as<double>(), T, part);
  }
  {
    ::bchar::ProfScope ps_("k_target_scale", s);
    k_target_scale<<<1, 256, 0, s>>>(part, kTargetBlocks, out);
  }
  {
    ::bchar::ProfScope ps_("k_cc_init", s);
    k_cc_init<<<blocks_for(n2, 256), 256, 0, s>>>(n2, lab);
  }
  BCHAR_HIP(hipGetLastError());
  // hook and compress until no label moves (each round that reports a
  // change lowered a label, so the rounds end)
  int rounds = 0;
  for (;; ++rounds) {
    BCHAR_REQUIRE(rounds < kMaxCcRounds, BCHAR_E_DEVICE,
                  "connected components of the transfer pattern did not settle");
    fill_i32(flag, 0, 1, s);
    {
      ::bchar::ProfScope ps_("k_cc_hook", s);
      k_cc_hook<<<blocks_for(n, 256), 256, 0, s>>>(row_ptr, col, n, lab, flag);
    }
    {
      ::bchar::ProfScope ps_("k_cc_compress", s);
      k_cc_compress<<<blocks_for(n2, 256), 256, 0, s>>>(n2, lab);
    }
    BCHAR_HIP(hipGetLastError());
    int32_t h = 0;
    BCHAR_HIP(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s));
    BCHAR_HIP(hipStreamSynchronize(s));
    if (h == 0) break;
  }
  fill_i32(flag + 1, 0, 1, s);
  {
    ::bchar::ProfScope ps_("k_cc_roots", s);
    k_cc_roots<<<blocks_for(n2, 256), 256, 0, s>>>(n2, lab, flag + 1);
  }
  BCHAR_HIP(hipGetLastError());
  TargetInfo info;
  double h[3];
  int32_t groups = 0;
  BCHAR_HIP(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
  BCHAR_HIP(hipMemcpyAsync(&groups, flag + 1, sizeof(groups), hipMemcpyDeviceToHost, s));
  BCHAR_HIP(hipStreamSynchronize(s));
  info.scale = h[2];
  info.groups = groups;
  BCHAR_REQUIRE(std::isfinite(h[2]) && h[2] > 0.0, BCHAR_E_INVALID_ARG,
                "non-solenoidal step: the tracked porous volumes do not sum to a positive "
                "finite value");
  if (groups == 1) {
    // one component: the whole domain's factor
    ::bchar::ProfScope ps_("k_scale_targets", s);
    k_scale_targets<<<blocks_for(n, 256), 256, 0, s>>>(n, T, nullptr, out + 2, b_row);
  } else {
    t->grp_ptr.reserve(sizeof(int32_t) * (n2 + 1));
    t->grp_perm.reserve(sizeof(int32_t) * n2);
    int32_t* ptr = t->grp_ptr.as<int32_t>();
    int32_t* perm = t->grp_perm.as<int32_t>();
    double* scale = ws.get<double>(n2);
    bucket_sort(lab, n2, n2, ptr, perm, ws, s);
    {
      ::bchar::ProfScope ps_("k_cc_scale", s);
      k_cc_scale<<<(unsigned)n2, 64, 0, s>>>(n, ptr, perm, T, m->b.as<double>(), scale);
    }
    {
      ::bchar::ProfScope ps_("k_scale_targets", s);
      k_scale_targets<<<blocks_for(n, 256), 256, 0, s>>>(n, T, lab, scale, b_row);
    }
  }
  BCHAR_HIP(hipGetLastError());
  BCHAR_HIP(hipStreamSynchronize(s));
  ws.rewind(mk);
  info.rounds = rounds + 1;
  return info;
}

// ---------------------------------------------------------------- lens

constexpr double kPi = 3.14159265358979323846;

// |B(r1) cap B(r2)| at centre distance d, 3D: the sphere lens
// pi (r1 + r2 - d)^2 (d^2 + 2 d (r1 + r2) - 3 (r1 - r2)^2) / (12 d).
template <class T>
__device__ __forceinline__ T sphere_lens(T r1, T r2, T d) {
  const T rmin = r1 < r2 ? r1 : r2;
  if (d <= fabs(r1 - r2)) return (T)(4.0 * kPi / 3.0) * rmin * rmin * rmin;
  const T sum = r1 + r2;
  if (d >= sum) return 0;
  const T g = sum - d;
  const T dr = r1 - r2;
  return (T)kPi * g * g * (d * d + (T)2 * d * sum - (T)3 * dr * dr) / ((T)12 * d);
}

// 2D: r1^2 a1 + r2^2 a2 - Delta / 2 with Delta = 2 d rho (rho the half
// chord) and the half-angles a_i taken by atan2 for accuracy.
template <class T>
__device__ __forceinline__ T disk_lens(T r1, T r2, T d) {
  const T rmin = r1 < r2 ? r1 : r2;
  if (d <= fabs(r1 - r2)) return (T)kPi * rmin * rmin;
  const T sum = r1 + r2;
  if (d >= sum) return 0;
  T p = (sum - d) * (d + r1 - r2) * (d - r1 + r2) * (d + sum);
  p = p > 0 ? p : 0;
  const T Delta = sqrt(p);
  const T a1 = atan2(Delta, d * d + r1 * r1 - r2 * r2);
  const T a2 = atan2(Delta, d * d + r2 * r2 - r1 * r1);
  const T v = r1 * r1 * a1 + r2 * r2 * a2 - (T)0.5 * Delta;
  return v > 0 ? v : 0;
}

template <int DIM, class T>
__device__ __forceinline__ T lens(T r1, T r2, T d) {
  return DIM == 3 ? sphere_lens<T>(r1, r2, d) : disk_lens<T>(r1, r2, d);
}

// ---------------------------------------------------------------- assembly

constexpr int kXcds = 8;         // accelerator complex dies of the MI355X
constexpr int kTileThreads = 256; // tracked balls per tile (one thread each)
constexpr int kTileCap = 2048;    // overlaps of one group of cells held in LDS
constexpr int kStash = 8;         // overlapping slots a thread remembers between passes
constexpr int kStageBalls = 1024;  // residing balls of a tile's search block staged in LDS
constexpr int kStageBuckets = 1280; // bucket starts of the block (buckets + rows)
constexpr int kStageRows = 256;    // bucket rows of the block

// flags of one assembly launch (int32, cleared before it)
enum {
  kFlagFirstVoid = 0,   // lowest tracked ball with S = 0 (INT32_MAX: none)
  kFlagVoidRows,        // tracked cells with a void ball
  kFlagCellOverflow,    // largest overlap count of a single cell beyond kTileCap
  kFlagEntries,         // staged entries beyond the tiles' own staging room
  kFlagPairs,           // candidate pairs (kept pairs only)
  kFlagStageOverflow,   // staging or pair storage too small
  kNumFlags
};

struct TileParams {
  int64_t n_cells, n_balls;
  int nbpc;                 // balls per cell, 0: variable (ball_ptr)
  const int32_t* ball_ptr;  // variable layouts: first ball of every cell, n_cells + 1
  const int32_t* tile_cell; // variable layouts: first cell of every tile, n_tiles + 1
  // Cartesian tiles: tx * ty * tz cells per tile, nt tiles per axis;
  // tx == 0: tiles are runs of cells_per_tile consecutive cells
  int tx, ty, tz;
  int64_t nt[3];
  int64_t n[3];
  int cells_per_tile;
  int64_t n_tiles;
  // hash
  int64_t nbk[3];
  double org[3];
  double inv_hs;
  double rmax;
  double r0;                // radius of every residing ball (uniform layouts)
  const double* rho;        // per cell
  const double* phi;        // per cell
  const double* bvol;       // per ball, |B_{K,s}|
  const double* lam;        // per ball log growth (non-solenoidal u), or null
  const uint8_t* ghost;     // per cell ghost flag, or null (no ghost cells)
  const double* tracked;    // dim * n_balls
  const double* r_hat;      // n_balls
  const int32_t* bucket_start;
  const double* bk_cen;     // dim * n_balls, bucket order
  const float* bk_cen32;
  const double* bk_rad;     // n_balls, bucket order
  const int32_t* bk_cell;   // residing cell of each slot
  const int32_t* bk_ball;   // residing ball of each slot
  const double* bk_w;       // rho_M phi_M of each slot
  // outputs
  int32_t* row_cnt;         // unique residing cells per row
  int32_t* stage_off;       // staging position of every row
  int32_t* stage_col;       // tile t stages at t * kTileCap, what does not fit
  double* stage_val;        // there at n_tiles * kTileCap + (atomic count)
  int64_t stage_cap;
  int32_t* tile_pairs;      // overlaps of every tile (pairs not kept)
  int lds_stage;            // stage each tile's search block in LDS when it fits
  int32_t* pair_a;          // may be null
  int32_t* pair_b;
  int64_t pair_cap;
  int32_t* flags;           // kNumFlags
};

// Block-wide exclusive scan of one int per thread (256 threads); *total is
// the sum over the block.
__device__ __forceinline__ int block_excl_scan(int v, int* s_wave, int& total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int incl = wave_incl_scan_i(v);
  if (lane == kWave - 1) s_wave[w] = incl;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kTileThreads / kWave; ++i) {
    const int x = s_wave[i];
    base += i < w ? x : 0;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return base + incl - v;
}

// Predicate ((dx*dx + dy*dy) + dz*dz) < (ra + rb)^2 (rs = ra + rb), rounded
// once per operation (no contraction into FMA) so that it is reproducible.
template <int DIM, class T>
__device__ __forceinline__ bool overlap(const T p[3], const T c[3], T rs, T& d2) {
#pragma clang fp contract(off)
  T dx = p[0] - c[0];
  T dy = p[1] - c[1];
  T s = dx * dx;
  s = s + dy * dy;
  if (DIM == 3) {
    T dz = p[2] - c[2];
    s = s + dz * dz;
  }
  d2 = s;
  return s < rs * rs;
}

// Every residing ball overlapping the tracked ball (p, ra): the buckets
// that can hold a centre within ra + r_max of p (the range widened by a
// relative 1e-6 so that binary32 rounding of the predicate cannot reach
// past it; the predicate alone decides), walked as rows of consecutive
// buckets along x, each row one run of slots.  f(slot, rb, d2).
template <int DIM, class T>
__device__ __forceinline__ void search_block(const TileParams& P, const T p[3], T ra,
                                             int64_t blo[3], int64_t side[3]) {
  const double D = ((double)ra + P.rmax) * (1.0 + 1e-6);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    blo[a] = 0;
    side[a] = 1;
  }
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const double x = (double)p[a] - P.org[a];
    int64_t lo = (int64_t)floor((x - D) * P.inv_hs);
    int64_t hi = (int64_t)floor((x + D) * P.inv_hs);
    lo = lo < 0 ? 0 : lo;
    hi = hi >= P.nbk[a] ? P.nbk[a] - 1 : hi;
    blo[a] = lo;
    side[a] = hi >= lo ? hi - lo + 1 : 0;
  }
}

template <int DIM, class T, bool UR, class F>
__device__ __forceinline__ void for_each_overlap(const TileParams& P, const T p[3], T ra, F&& f) {
  int64_t blo[3], side[3];
  search_block<DIM, T>(P, p, ra, blo, side);
  const int64_t nb = P.n_balls;
  for (int64_t bz = 0; bz < side[2]; ++bz)
    for (int64_t by = 0; by < side[1]; ++by) {
      const int64_t row = blo[0] + P.nbk[0] * ((blo[1] + by) + P.nbk[1] * (blo[2] + bz));
      const int32_t lo = P.bucket_start[row];
      const int32_t hi = P.bucket_start[row + side[0]];
      for (int32_t e = lo; e < hi; ++e) {
        T c[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < DIM; ++a)
          c[a] = sizeof(T) == 8 ? (T)P.bk_cen[a * nb + e] : (T)P.bk_cen32[a * nb + e];
        const T rb = UR ? (T)P.r0 : (T)P.bk_rad[e];
        T d2;
        if (overlap<DIM, T>(p, c, ra + rb, d2)) f(e, rb, d2);
      }
    }
}

// Cell of local index lc in tile t, or -1 past the mesh.
__device__ __forceinline__ int64_t tile_cell_id(const TileParams& P, int64_t t, int lc) {
  if (P.tile_cell) {
    const int64_t K = (int64_t)P.tile_cell[t] + lc;
    return K < P.tile_cell[t + 1] ? K : -1;
  }
  if (P.tx == 0) {
    const int64_t K = t * P.cells_per_tile + lc;
    return K < P.n_cells ? K : -1;
  }
  const int lx = lc % P.tx, ly = (lc / P.tx) % P.ty, lz = lc / (P.tx * P.ty);
  const int64_t i = (t % P.nt[0]) * P.tx + lx;
  const int64_t j = ((t / P.nt[0]) % P.nt[1]) * P.ty + ly;
  const int64_t k = (t / (P.nt[0] * P.nt[1])) * P.tz + lz;
  if (i >= P.n[0] || j >= P.n[1] || k >= P.n[2]) return -1;
  return i + P.n[0] * (j + P.n[1] * k);
}

// LDS of the assembly: the residing balls of the tile's search block
// (staged for pass 1) share their room with the merge arrays (pass 2 on)
// (STG false: no staging, the smaller footprint lets more workgroups share
// a CU)
template <int DIM, class T, bool UR, bool STG>
struct StageLayout {
  static constexpr int kBytesBall = DIM * (int)sizeof(T) + (UR ? 0 : (int)sizeof(T)) + 4;
  static constexpr int kStageBytes = STG ? kStageBalls * kBytesBall + 4 * kStageBuckets : 0;
  static constexpr int kMergeBytes = kTileCap * (4 + 8 + 1);
  static constexpr int kBytes = kStageBytes > kMergeBytes ? kStageBytes : kMergeBytes;
};

template <int DIM, class T, bool UR, bool STG>
__global__ void __launch_bounds__(kTileThreads) k_assemble(TileParams P) {
  using L = StageLayout<DIM, T, UR, STG>;
  __shared__ __align__(16) unsigned char s_union[L::kBytes];
  // merge view
  double* const s_val = reinterpret_cast<double*>(s_union);
  int32_t* const s_key = reinterpret_cast<int32_t*>(s_union + 8 * kTileCap);
  uint8_t* const s_first = s_union + 12 * kTileCap;
  // staging view: coordinates (SoA), radii, global slot, local bucket starts
  T* const g_cen = reinterpret_cast<T*>(s_union);
  T* const g_rad = g_cen + DIM * kStageBalls;
  int32_t* const g_slot =
      reinterpret_cast<int32_t*>(s_union + (DIM + (UR ? 0 : 1)) * sizeof(T) * kStageBalls);
  int32_t* const g_bst = g_slot + kStageBalls;
  __shared__ int32_t s_box[8];                     // block lo (3), hi (3)
  __shared__ int32_t s_rowoff[kStageRows + 1];     // local slot offset of every block row
  __shared__ int32_t s_rowg0[kStageRows];          // its first global slot
  __shared__ int32_t s_cstart[kTileThreads + 1];   // first overlap of every local cell
  __shared__ int32_t s_ucnt[kTileThreads];         // unique residing cells of every local cell
  __shared__ int32_t s_upre[kTileThreads];         // their exclusive scan within the group
  __shared__ int32_t s_wave[kTileThreads / kWave];
  __shared__ int32_t s_misc[5];
  __shared__ int32_t s_stash[kStash * kTileThreads];   // slot i of thread j at i * 256 + j

  // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, each
  // with its own L2; XCD j takes the j-th contiguous chunk of tiles so that
  // neighbouring tiles, which read the same hash buckets, share an L2
  const int64_t chunk = (P.n_tiles + kXcds - 1) / kXcds;
  const int64_t t = (int64_t)(blockIdx.x % kXcds) * chunk + blockIdx.x / kXcds;
  if (t >= P.n_tiles) return;   // the whole block leaves together
  const int tid = threadIdx.x;
  const int64_t nb = P.n_balls;

  // ---- this thread's tracked ball: local cell lc (every thread of a
  // uniform layout has one, also past the mesh), ball b (-1: none), its rank
  // s in the cell and the cell's ball count nbc
  int lc = -1, s = 0, nbc = 1;
  int64_t K = -1, b = -1;
  int nct = 0;   // local cells of the tile
  if (P.nbpc > 0) {
    nct = kTileThreads / P.nbpc;
    if (tid < nct * P.nbpc) {
      lc = tid / P.nbpc;
      s = tid % P.nbpc;
      nbc = P.nbpc;
      K = tile_cell_id(P, t, lc);
      if (K >= 0) b = K * P.nbpc + s;
    }
  } else {
    const int64_t c0 = P.tile_cell[t], c1 = P.tile_cell[t + 1];
    nct = (int)(c1 - c0);
    const int64_t bb = (int64_t)P.ball_ptr[c0] + tid;
    if (bb < P.ball_ptr[c1]) {
      // the cell holding ball bb: binary search over the tile's cells
      int64_t lo = c0, hi = c1 - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (P.ball_ptr[mid] <= bb) lo = mid;
        else hi = mid - 1;
      }
      K = lo;
      lc = (int)(K - c0);
      b = bb;
      s = (int)(bb - P.ball_ptr[K]);
      nbc = P.ball_ptr[K + 1] - P.ball_ptr[K];
    }
  }

  T p[3] = {0, 0, 0};
  T ra = 0;
  double mass = 0.0;
  if (b >= 0) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) p[a] = (T)P.tracked[a * nb + b];
    ra = (T)P.r_hat[b];
    mass = P.rho[K] * P.phi[K] * P.bvol[b];   // rho_K phi_K |B_{K,s}|
    // non-solenoidal u: times exp(lam), the Liouville growth of the ball
    if (P.lam) mass = mass * exp(P.lam[b]);
  }

  // ---- the search block of the whole tile: the union of its balls'
  // bucket blocks (each ball's block as for_each_overlap computes it)
  int64_t blo[3] = {0, 0, 0}, side[3] = {1, 1, 1};
  int32_t bl[3] = {0, 0, 0}, bn[3] = {1, 1, 1};
  bool staged = false;
  if constexpr (STG) {
  if (tid < 8) s_box[tid] = tid < 3 ? INT32_MAX : (tid < 6 ? -1 : 0);
  __syncthreads();
  if (b >= 0) {
    search_block<DIM, T>(P, p, ra, blo, side);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      atomicMin(&s_box[a], (int32_t)blo[a]);
      atomicMax(&s_box[3 + a], (int32_t)(blo[a] + side[a] - 1));
    }
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    bl[a] = s_box[a];
    bn[a] = s_box[3 + a] - s_box[a] + 1;
  }
  // rows of buckets along x in the block, each a run of slots
  const int nrows = bn[0] > 0 ? bn[1] * bn[2] : 0;
  staged = nrows > 0 && nrows <= kStageRows &&
                nrows * (bn[0] + 1) <= kStageBuckets;
  if (staged) {
    // one row per thread (nrows <= 256): its slots, scanned over the block
    int n_r = 0;
    if (tid < nrows) {
      const int64_t row =
          bl[0] + P.nbk[0] * ((bl[1] + tid % bn[1]) + P.nbk[1] * (bl[2] + tid / bn[1]));
      const int32_t g0 = P.bucket_start[row];
      s_rowg0[tid] = g0;
      n_r = P.bucket_start[row + bn[0]] - g0;
    }
    int total_slots = 0;
    const int ro = block_excl_scan(n_r, s_wave, total_slots);
    if (tid < nrows) s_rowoff[tid] = ro;
    if (tid == 0) s_rowoff[nrows] = total_slots;
    __syncthreads();
    staged = total_slots <= kStageBalls;   // the same on every thread
  }
  if (staged) {
    // local bucket starts of every row, then the slots of all rows, both
    // spread over the threads
    const int nx1 = bn[0] + 1;
    for (int q = tid; q < nrows * nx1; q += kTileThreads) {
      const int r = q / nx1, i = q % nx1;
      const int64_t row = bl[0] + P.nbk[0] * ((bl[1] + r % bn[1]) + P.nbk[1] * (bl[2] + r / bn[1]));
      g_bst[q] = s_rowoff[r] + (P.bucket_start[row + i] - s_rowg0[r]);
    }
    const int total = s_rowoff[nrows];
    for (int l = tid; l < total; l += kTileThreads) {
      // the row holding local slot l: the last r with s_rowoff[r] <= l
      int lo = 0, hi = nrows - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (s_rowoff[mid] <= l) lo = mid;
        else hi = mid - 1;
      }
      const int32_t e = s_rowg0[lo] + (l - s_rowoff[lo]);
#pragma unroll
      for (int a = 0; a < DIM; ++a)
        g_cen[a * kStageBalls + l] =
            sizeof(T) == 8 ? (T)P.bk_cen[a * nb + e] : (T)P.bk_cen32[a * nb + e];
      if (!UR) g_rad[l] = (T)P.bk_rad[e];
      g_slot[l] = e;
    }
    __syncthreads();
  }
  }  // STG

  // ---- pass 1: number of overlaps and S = sum omega, in slot order
  int cnt = 0;
  double S = 0.0;
  auto count = [&](int32_t e, T rb, T d2) {
    S += P.bk_w[e] * (double)lens<DIM, T>(ra, rb, sqrt(d2));
    if (cnt < kStash) s_stash[cnt * kTileThreads + tid] = e;
    ++cnt;
  };
  if (b >= 0 && staged) {
    // the same rows and slots as for_each_overlap, read from LDS
    for (int64_t bz = 0; bz < side[2]; ++bz)
      for (int64_t by = 0; by < side[1]; ++by) {
        const int r = (int)((blo[1] + by - bl[1]) + bn[1] * (blo[2] + bz - bl[2]));
        const int x0 = (int)(blo[0] - bl[0]);
        const int lo = g_bst[r * (bn[0] + 1) + x0], hi = g_bst[r * (bn[0] + 1) + x0 + side[0]];
        for (int l = lo; l < hi; ++l) {
          T c[3] = {0, 0, 0};
#pragma unroll
          for (int a = 0; a < DIM; ++a) c[a] = g_cen[a * kStageBalls + l];
          const T rb = UR ? (T)P.r0 : g_rad[l];
          T d2;
          if (overlap<DIM, T>(p, c, ra + rb, d2)) count(g_slot[l], rb, d2);
        }
      }
  } else if (b >= 0) {
    for_each_overlap<DIM, T, UR>(P, p, ra, count);
  }
  __syncthreads();   // the staged block is dead from here on (merge arrays share its room)
  s_ucnt[tid] = 0;   // void marks of the local cells until the scan below
  __syncthreads();
  // a ghost cell's ball that meets nothing carries its mass out of the
  // problem: no void
  if (b >= 0 && !(S > 0.0) && !(P.ghost && P.ghost[K])) {
    atomicMin(&P.flags[kFlagFirstVoid], (int32_t)b);
    atomicOr(&s_ucnt[lc], 1);
  }
  const double share = S > 0.0 ? mass / S : 0.0;

  // the balls of a cell are consecutive threads, so the block scan of the
  // counts gives every ball's first slot and every cell's range
  int H = 0;
  const int off = block_excl_scan(cnt, s_wave, H);
  if (lc >= 0) {
    if (s == 0) s_cstart[lc] = off;
    if (s == nbc - 1) s_cstart[lc + 1] = off + cnt;
    if (s == 0 && b >= 0 && s_ucnt[lc]) atomicAdd(&P.flags[kFlagVoidRows], 1);
  }
  if (tid == 0) {
    // kept pairs reserve their room with an atomic add; otherwise only
    // their number is written, per tile
    if (P.pair_a) {
      s_misc[0] = atomicAdd(&P.flags[kFlagPairs], H);
      if ((int64_t)s_misc[0] + H > P.pair_cap) atomicOr(&P.flags[kFlagStageOverflow], 1);
    } else {
      s_misc[0] = 0;
      P.tile_pairs[t] = H;
    }
    s_misc[3] = 0;   // staging entries used in the tile's own room
  }
  __syncthreads();
  const int pbase = s_misc[0];
  const bool write_pairs = P.pair_a && (int64_t)pbase + H <= P.pair_cap;

  // ---- groups of whole cells whose overlaps fit in LDS (one group unless
  // the tile overlaps more than kTileCap residing balls)
  int gs = 0;
  while (gs < nct) {
    // the group is cells gs .. ge-1, the longest run from gs that fits
    // (cell starts are non-decreasing in the local index)
    if (tid == 0) s_misc[1] = gs;
    __syncthreads();
    if (tid >= gs && tid < nct && s_cstart[tid + 1] - s_cstart[gs] <= kTileCap)
      atomicMax(&s_misc[1], tid + 1);
    __syncthreads();
    const int ge = s_misc[1];
    const int gbase = s_cstart[gs];
    if (ge == gs) {
      // one cell alone overlaps more residing balls than LDS holds
      if (tid == 0) atomicMax(&P.flags[kFlagCellOverflow], s_cstart[gs + 1] - gbase);
      __syncthreads();
      gs = gs + 1;
      continue;
    }
    const bool mine = b >= 0 && lc >= gs && lc < ge;
    // pass 2: the same overlaps again, written in order: from the slots
    // remembered in pass 1, or (more than kStash) by walking the buckets
    if (mine) {
      int o = off - gbase;
      int po = pbase + off;
      auto put = [&](int32_t e, T rb, T d2) {
        const double om = P.bk_w[e] * (double)lens<DIM, T>(ra, rb, sqrt(d2));
        s_key[o] = P.bk_cell[e];
        s_val[o] = share * om;
        ++o;
        if (write_pairs) {
          P.pair_a[po] = (int32_t)b;
          P.pair_b[po] = P.bk_ball[e];
          ++po;
        }
      };
      if (cnt <= kStash) {
        for (int i = 0; i < cnt; ++i) {
          const int32_t e = s_stash[i * kTileThreads + tid];
          T c[3] = {0, 0, 0};
#pragma unroll
          for (int a = 0; a < DIM; ++a)
            c[a] = sizeof(T) == 8 ? (T)P.bk_cen[a * nb + e] : (T)P.bk_cen32[a * nb + e];
          const T rb = UR ? (T)P.r0 : (T)P.bk_rad[e];
          T d2;
          overlap<DIM, T>(p, c, ra + rb, d2);
          put(e, rb, d2);
        }
      } else {
        for_each_overlap<DIM, T, UR>(P, p, ra, put);
      }
    }
    s_ucnt[tid] = 0;
    __syncthreads();
    // first occurrence of every residing cell within its tracked cell
    int e0 = 0, e1 = 0;
    if (mine) {
      e0 = s_cstart[lc] - gbase;
      e1 = s_cstart[lc + 1] - gbase;
      int u = 0;
      for (int e = e0 + s; e < e1; e += nbc) {
        const int32_t k = s_key[e];
        int first = 1;
        for (int j = e0; j < e; ++j)
          if (s_key[j] == k) {
            first = 0;
            break;
          }
        s_first[e] = (uint8_t)first;
        u += first;
      }
      if (u) atomicAdd(&s_ucnt[lc], u);
    }
    __syncthreads();
    // unique counts scanned over the group's cells; the group stages in
    // the tile's own room while it lasts, else reserves room at the end
    // of the staging array with one atomic add
    int U = 0;
    const int uc = (tid >= gs && tid < ge) ? s_ucnt[tid] : 0;
    const int uo = block_excl_scan(uc, s_wave, U);
    if (tid >= gs && tid < ge) s_upre[tid] = uo;
    if (tid == 0) {
      const int used = s_misc[3];
      if (used + U <= kTileCap) {
        s_misc[2] = used;
        s_misc[3] = used + U;
        s_misc[4] = 0;
      } else {
        s_misc[2] = atomicAdd(&P.flags[kFlagEntries], U);
        s_misc[4] = 1;
      }
    }
    __syncthreads();
    const int64_t sbase = s_misc[4] ? P.n_tiles * kTileCap + s_misc[2]
                                    : t * kTileCap + s_misc[2];
    if (sbase + U > P.stage_cap) {
      if (tid == 0) atomicOr(&P.flags[kFlagStageOverflow], 1);
    } else if (mine) {
      const int64_t rbase = sbase + s_upre[lc];
      for (int e = e0 + s; e < e1; e += nbc) {
        if (!s_first[e]) continue;
        const int32_t k = s_key[e];
        int rank = 0;
        double v = 0.0;
        for (int j = e0; j < e1; ++j) {
          const int32_t kj = s_key[j];
          if (s_first[j] && kj < k) ++rank;
          if (kj == k) v += s_val[j];
        }
        P.stage_col[rbase + rank] = k;
        P.stage_val[rbase + rank] = v;
      }
      if (s == 0) {
        P.row_cnt[K] = s_ucnt[lc];
        P.stage_off[K] = (int32_t)rbase;
      }
    }
    __syncthreads();
    gs = ge;
  }
}

// Rows laid out as CSR: row K's entries move from its staging position to
// row_ptr[K] (one thread per row).
__global__ void k_scatter_rows(int64_t n_cells, const int32_t* __restrict__ row_ptr,
                               const int32_t* __restrict__ stage_off,
                               const int32_t* __restrict__ stage_col,
                               const double* __restrict__ stage_val, int32_t* __restrict__ col,
                               double* __restrict__ val) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= n_cells) return;
  const int32_t d = row_ptr[K], n = row_ptr[K + 1] - d;
  const int32_t so = stage_off[K];
  for (int32_t i = 0; i < n; ++i) {
    col[d + i] = stage_col[so + i];
    val[d + i] = stage_val[so + i];
  }
}

__global__ void k_init_flags(int32_t* __restrict__ f) {
  const int i = threadIdx.x;
  if (i < kNumFlags) f[i] = i == kFlagFirstVoid ? INT32_MAX : 0;
}

template <int DIM, class T>
static void launch_assemble_t(const TileParams& P, unsigned grid, bool ur, hipStream_t s) {
  ::bchar::ProfScope ps_("k_assemble", s);
  if (P.lds_stage) {
    if (ur)
      k_assemble<DIM, T, true, true><<<grid, kTileThreads, 0, s>>>(P);
    else
      k_assemble<DIM, T, false, true><<<grid, kTileThreads, 0, s>>>(P);
  } else {
    if (ur)
      k_assemble<DIM, T, true, false><<<grid, kTileThreads, 0, s>>>(P);
    else
      k_assemble<DIM, T, false, false><<<grid, kTileThreads, 0, s>>>(P);
  }
}

static void launch_assemble(int dim, int precision, const TileParams& P, bool ur, hipStream_t s) {
  const unsigned grid = (unsigned)(((P.n_tiles + kXcds - 1) / kXcds) * kXcds);
  const bool f32 = precision != BCHAR_FP64;
  if (dim == 2) {
    if (f32) launch_assemble_t<2, float>(P, grid, ur, s);
    else launch_assemble_t<2, double>(P, grid, ur, s);
  } else {
    if (f32) launch_assemble_t<3, float>(P, grid, ur, s);
    else launch_assemble_t<3, double>(P, grid, ur, s);
  }
  BCHAR_HIP(hipGetLastError());
}

// Tile shape of a uniform layout: a block of cells on a Cartesian mesh
// (square-ish in the plane, so that the tile's tracked balls read few
// hash rows), a run of consecutive cells otherwise.
// Cartesian tiles of kTileThreads / nbpc cells: the most cubic power-of-
// two box (256 cells -> 8x8x4, 32 -> 4x4x2; 2D 64 -> 8x8), or with
// aspect a != 0 the last axis's extent divided (a > 0) or multiplied
// (a < 0) by 2^|a|, the others refitted (32 cells: a = 1 -> 8x4x1,
// a = -1 -> 4x2x4).  Rows come out in cell order whatever the shape.
static void tile_shape(const bchar_mesh_s* m, int aspect, TileParams& P) {
  P.cells_per_tile = kTileThreads / m->nbpc;
  P.tx = P.ty = P.tz = 0;
  for (int a = 0; a < 3; ++a) {
    P.n[a] = m->n[a];
    P.nt[a] = 1;
  }
  if (m->kind == BCHAR_MESH_CARTESIAN) {
    const int c = P.cells_per_tile;
    auto shifted = [&](int e) {
      for (int k = 0; k < aspect && e > 1; ++k) e /= 2;
      for (int k = 0; k < -aspect && e < c; ++k) e *= 2;
      return e;
    };
    if (m->dim == 3) {
      int tz = 1;
      while (tz * tz * tz * 4 < c) tz *= 2;
      tz = shifted(tz);
      const int txy = c / tz;
      int tx = 1;
      while (tx * tx < txy) tx *= 2;
      P.tx = tx;
      P.ty = txy / tx;
      P.tz = tz;
    } else {
      int ty = 1;
      while (ty * ty < c) ty *= 2;
      ty = shifted(c / ty);
      P.ty = ty;
      P.tx = c / ty;
      P.tz = 1;
    }
    const int t3[3] = {P.tx, P.ty, P.tz};
    P.n_tiles = 1;
    for (int a = 0; a < 3; ++a) {
      P.nt[a] = (m->n[a] + t3[a] - 1) / t3[a];
      P.n_tiles *= P.nt[a];
    }
  } else {
    P.n_tiles = (m->n_cells + P.cells_per_tile - 1) / P.cells_per_tile;
  }
}

bchar_status assemble_v(bchar_mesh_s* m, const double* tracked, const double* r_hat,
                        const double* lam, int precision, bool keep_pairs, bool lds_stage,
                        int tile_aspect, bchar_transfer_s* t, int64_t* first_void,
                        hipStream_t s) {
  Arena& ws = t->ws;
  const int64_t nc = m->n_cells;
  TileParams P{};
  P.n_cells = nc;
  P.n_balls = m->n_balls;
  P.nbpc = m->nbpc;
  if (m->nbpc > 0) {
    tile_shape(m, tile_aspect, P);
  } else {
    P.ball_ptr = m->ball_ptr.as<int32_t>();
    P.tile_cell = m->tile_cell.as<int32_t>();
    P.n_tiles = m->n_tiles;
  }
  for (int a = 0; a < 3; ++a) {
    P.nbk[a] = m->nbk[a];
    P.org[a] = m->box_lo[a];
  }
  P.inv_hs = 1.0 / m->hs;
  P.rmax = m->rmax;
  P.r0 = m->r0;
  P.lds_stage = lds_stage ? 1 : 0;
  P.rho = m->rho.as<double>();
  P.phi = m->phi.as<double>();
  P.bvol = m->bvol.as<double>();
  P.lam = lam;
  P.ghost = m->ghost.as<uint8_t>();
  P.tracked = tracked;
  P.r_hat = r_hat;
  P.bucket_start = m->bucket_start.as<int32_t>();
  P.bk_cen = m->bk_cen.as<double>();
  P.bk_cen32 = m->bk_cen32.as<float>();
  P.bk_rad = m->bk_rad.as<double>();
  P.bk_cell = m->bk_cell.as<int32_t>();
  P.bk_ball = m->bk_ball.as<int32_t>();
  P.bk_w = m->bk_w.as<double>();
  P.row_cnt = ws.get<int32_t>(nc + 1);
  P.stage_off = ws.get<int32_t>(nc + 1);
  P.flags = ws.get<int32_t>(kNumFlags);
  P.tile_pairs = ws.get<int32_t>(P.n_tiles + 1);
  int32_t* pair_sum = ws.get<int32_t>(P.n_tiles + 1);
  // staging: every tile's own room of kTileCap entries, then room for the
  // groups that do not fit there (the last build's need, at least 1024); a
  // launch that finds it too small is repeated with what it needed
  const int64_t own = P.n_tiles * kTileCap;
  int64_t cap_e = own + std::max<int64_t>(t->stage_need, 1024);
  int64_t cap_p = keep_pairs ? std::max<int64_t>(t->pair_need, 16 * m->n_balls + 1024) : 0;
  int32_t hf[kNumFlags];
  int32_t npairs_tiles = 0;
  for (int attempt = 0;; ++attempt) {
    t->stage_col.reserve(sizeof(int32_t) * cap_e);
    t->stage_val.reserve(sizeof(double) * cap_e);
    P.stage_col = t->stage_col.as<int32_t>();
    P.stage_val = t->stage_val.as<double>();
    P.stage_cap = cap_e;
    P.pair_a = P.pair_b = nullptr;
    P.pair_cap = 0;
    if (keep_pairs) {
      t->pair_a.reserve(sizeof(int32_t) * cap_p);
      t->pair_b.reserve(sizeof(int32_t) * cap_p);
      P.pair_a = t->pair_a.as<int32_t>();
      P.pair_b = t->pair_b.as<int32_t>();
      P.pair_cap = cap_p;
    }
    k_init_flags<<<1, 64, 0, s>>>(P.flags);
    BCHAR_HIP(hipGetLastError());
    launch_assemble(m->dim, precision, P, m->r_uniform, s);
    if (!keep_pairs) {
      // the number of pairs: the tiles' counts summed (the scan's total)
      exclusive_scan_i32_async(P.tile_pairs, pair_sum, P.n_tiles, ws, s);
      BCHAR_HIP(hipMemcpyAsync(&npairs_tiles, pair_sum + P.n_tiles, sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
    }
    BCHAR_HIP(hipMemcpyAsync(hf, P.flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    BCHAR_HIP(hipStreamSynchronize(s));
    t->n_void_rows = hf[kFlagVoidRows];
    if (hf[kFlagCellOverflow] > 0)
      throw Error{BCHAR_E_UNSUPPORTED, "a tracked cell overlaps " +
                                           std::to_string(hf[kFlagCellOverflow]) +
                                           " residing balls (more than " +
                                           std::to_string(kTileCap) + ")"};
    if (hf[kFlagFirstVoid] != INT32_MAX) {
      *first_void = hf[kFlagFirstVoid];
      return BCHAR_E_VOID_ROW;
    }
    if (!hf[kFlagStageOverflow]) break;
    BCHAR_REQUIRE(attempt == 0, BCHAR_E_DEVICE, "assembly staging still too small");
    cap_e = std::max<int64_t>(cap_e, own + (int64_t)hf[kFlagEntries] + hf[kFlagEntries] / 4 +
                                         1024);
    if (keep_pairs)
      cap_p = std::max<int64_t>(cap_p, (int64_t)hf[kFlagPairs] + hf[kFlagPairs] / 4 + 1024);
  }
  t->stage_need = std::max<int64_t>(t->stage_need, (int64_t)hf[kFlagEntries] +
                                                         hf[kFlagEntries] / 4);
  if (keep_pairs)
    t->pair_need = std::max<int64_t>(t->pair_need, (int64_t)hf[kFlagPairs] + hf[kFlagPairs] / 4 +
                                                       1024);
  t->row_ptr.reserve(sizeof(int32_t) * (nc + 1));
  int32_t* row_ptr = t->row_ptr.as<int32_t>();
  const int64_t nnz = exclusive_scan_i32(P.row_cnt, row_ptr, nc, ws, s);
  t->nnz = nnz;
  t->n_pairs = keep_pairs ? hf[kFlagPairs] : npairs_tiles;
  t->col.reserve(sizeof(int32_t) * (nnz + 1));
  t->V.reserve(sizeof(double) * (nnz + 1));
  {
    ::bchar::ProfScope ps_("k_scatter_rows", s);
    k_scatter_rows<<<blocks_for(nc, 256), 256, 0, s>>>(nc, row_ptr, P.stage_off,
                                                      P.stage_col, P.stage_val,
                                                      t->col.as<int32_t>(), t->V.as<double>());
  }
  BCHAR_HIP(hipGetLastError());
  return BCHAR_OK;
}

}  // namespace bchar
