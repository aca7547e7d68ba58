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
// assemble: one wavefront per tracked cell K.  Lanes are split into
//          n_balls_per_cell groups; the lanes of a group share the 3^d (or
//          (2w+1)^d) hash buckets around that ball's tracked centre.  For
//          every overlapping residing ball (predicate without sqrt or FMA,
//          tangency excluded) the weight omega = rho_M phi_M |B_hat cap B|
//          is formed; the group reduces S = sum omega; the shares
//          rho_K phi_K |B| omega / S are compacted into LDS in a fixed
//          order and merged by residing cell M.  A count pass gives the row
//          lengths, a scan gives row_ptr, and a fill pass (same arithmetic)
//          writes sorted columns and values.  No floating-point atomics: the
//          result does not depend on scheduling.
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
  // centroids (ball centres, SoA), the domain box and the location grid
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

// Multilinear interpolation, written as the sum over the 2^d lattice
// corners of (product of the per-axis weights f or 1 - f) times the nodal
// value, corners in binary order, axes in order.  The query is clamped into
// the lattice box, t = (q - origin) / spacing, the lattice cell is
// floor(t) clamped to [0, m - 2].  Every operation is rounded on its own (no
// contraction), so that binary64 tracking is reproducible operation by
// operation.
template <int DIM, class T>
__device__ __forceinline__ void q1(const VelocityView<T>& V, const T x[3], T out[3]) {
#pragma clang fp contract(off)
  int64_t idx[3] = {0, 0, 0};
  T f[3] = {0, 0, 0};
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

// v = u / phi, phi of the cell containing x (floor((x - origin) / h),
// clamped), or the common value when phi is constant.
template <int DIM, class T>
__device__ __forceinline__ void speed(const VelocityView<T>& V, const PhiView<T>& P,
                                      const T x[3], T v[3]) {
#pragma clang fp contract(off)
  q1<DIM, T>(V, x, v);
  T ph;
  if (P.constant) {
    ph = P.phi0;
  } else if (P.simplex) {
    // the cell of x clamped into the domain box
    double q[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const double xa = (double)x[a];
      q[a] = xa < P.box_lo[a] ? P.box_lo[a] : (xa > P.box_hi[a] ? P.box_hi[a] : xa);
    }
    ph = (T)P.phi[locate<DIM, T>(P, q)];
  } else {
    int64_t cid = 0, stride = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      int64_t i = (int64_t)floor((x[a] - P.org[a]) / P.h[a]);
      i = i < 0 ? 0 : (i >= P.n[a] ? P.n[a] - 1 : i);
      cid += i * stride;
      stride *= P.n[a];
    }
    ph = (T)P.phi[cid];
  }
#pragma unroll
  for (int a = 0; a < DIM; ++a) v[a] = v[a] / ph;
}

// One classical RK4 step per sub-interval, backward: stage points
// X - (tau/2) k1, X - (tau/2) k2, X - tau k3, update
// X - (tau/6) (((k1 + 2 k2) + 2 k3) + k4), then clamp into the box.
template <int DIM, class T>
__device__ __forceinline__ void rk4_back(const VelocityView<T>& V, const PhiView<T>& P, T X[3],
                                         T tau, int substeps, const T lo[3], const T hi[3]) {
#pragma clang fp contract(off)
  const T htau = (T)0.5 * tau;
  const T tau6 = tau / (T)6;
  for (int st = 0; st < substeps; ++st) {
    T k1[3], k2[3], k3[3], k4[3], y[3];
    speed<DIM, T>(V, P, X, k1);
#pragma unroll
    for (int a = 0; a < DIM; ++a) y[a] = X[a] - htau * k1[a];
    speed<DIM, T>(V, P, y, k2);
#pragma unroll
    for (int a = 0; a < DIM; ++a) y[a] = X[a] - htau * k2[a];
    speed<DIM, T>(V, P, y, k3);
#pragma unroll
    for (int a = 0; a < DIM; ++a) y[a] = X[a] - tau * k3[a];
    speed<DIM, T>(V, P, y, k4);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      T acc = k1[a] + (T)2 * k2[a];
      acc = acc + (T)2 * k3[a];
      acc = acc + k4[a];
      T xa = X[a] - tau6 * acc;
      xa = xa > lo[a] ? xa : lo[a];
      X[a] = xa < hi[a] ? xa : hi[a];
    }
  }
}

template <int DIM, class T>
__global__ void k_trace(VelocityView<T> V, PhiView<T> P, const double* __restrict__ cen,
                        const double* __restrict__ rad, int64_t n_balls, T tau, int substeps,
                        T lo0, T lo1, T lo2, T hi0, T hi1, T hi2, double* __restrict__ tracked,
                        double* __restrict__ r_hat) {
#pragma clang fp contract(off)
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_balls) return;
  const T lo[3] = {lo0, lo1, lo2};
  const T hi[3] = {hi0, hi1, hi2};
  T C[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) C[a] = (T)cen[a * n_balls + b];
  T X[3] = {C[0], C[1], C[2]};
  rk4_back<DIM, T>(V, P, X, tau, substeps, lo, hi);
#pragma unroll
  for (int a = 0; a < DIM; ++a) tracked[a * n_balls + b] = (double)X[a];
  const T r = (T)rad[b];
  if (P.constant) {
    r_hat[b] = (double)r;
    return;
  }
  // eq. rTrackedBall: mean distance of the tracked cardinal points C +- r e_a
  T acc = 0;
  for (int a = 0; a < DIM; ++a) {
    for (int sg = 0; sg < 2; ++sg) {
      T Y[3] = {C[0], C[1], C[2]};
      Y[a] = sg == 0 ? Y[a] + r : Y[a] - r;
      rk4_back<DIM, T>(V, P, Y, tau, substeps, lo, hi);
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
                         hipStream_t s) {
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
  P.cen = m->cen.as<double>();
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
    k_trace<DIM, T><<<blocks_for(m->n_balls, 128), 128, 0, s>>>(
        V, P, m->cen.as<double>(), m->rad.as<double>(), m->n_balls, tau, substeps, lo[0], lo[1],
        lo[2], hi[0], hi[1], hi[2], tracked, r_hat);
  }
  BCHAR_HIP(hipGetLastError());
}

void trace_balls(const bchar_mesh_s* m, const bchar_velocity& u, double dt, int substeps,
                 int precision, double* tracked, double* r_hat, Arena& ws, hipStream_t s) {
  // With a porosity that varies from cell to cell the speed u/phi jumps on
  // cell faces, and the cardinal points of a ball start on faces: binary32
  // rounding would pick the neighbouring cell's phi.  Those meshes are
  // tracked in binary64 in both modes.
  if (precision == BCHAR_FP64 || !m->phi_const) {
    const double* comps[3] = {u.u[0], u.u[1], u.u[2]};
    if (m->dim == 2)
      launch_trace<2, double>(m, u, dt, substeps, comps, tracked, r_hat, s);
    else
      launch_trace<3, double>(m, u, dt, substeps, comps, tracked, r_hat, s);
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
      launch_trace<2, float>(m, u, dt, substeps, comps, tracked, r_hat, s);
    else
      launch_trace<3, float>(m, u, dt, substeps, comps, tracked, r_hat, s);
  }
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

constexpr int kCap = 1024;   // candidate shares per tracked cell held in LDS
constexpr int kXcds = 8;     // accelerator complex dies of the MI355X

// one workgroup per cell, padded to a multiple of the XCD count
static inline int64_t xcd_grid(int64_t n_cells) {
  return ((n_cells + kXcds - 1) / kXcds) * kXcds;
}

struct AsmParams {
  int64_t n_cells, n_balls;
  int nbpc;
  int64_t nbk[3];
  double org[3];
  double inv_hs;
  double hs;
  double rmax;            // largest residing radius
  const double* rho;      // per cell, porous density
  const double* bvol;     // per ball, |B_{K,s}|
  const double* phi;      // per cell
  const double* tracked;  // dim * n_balls
  const double* r_hat;    // n_balls
  const int32_t* bucket_start;
  const double* bk_cen;   // dim * n_balls, bucket order
  const float* bk_cen32;
  const int32_t* bk_ball;
  const double* bk_rad;   // n_balls, bucket order
  // outputs
  int32_t* row_cnt;       // count pass: unique M per row
  int32_t* pair_cnt;      // count pass: pairs per row
  const int32_t* row_ptr; // fill pass
  const int32_t* pair_ptr;
  int32_t* col;
  double* val;
  int32_t* pair_a;        // may be null
  int32_t* pair_b;
  int32_t* flags;         // [0] first void ball (min), [1] overflow
};

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

template <int DIM, class T>
__device__ __forceinline__ void search_range(const AsmParams& P, const T p[3], double reach,
                                             int64_t blo[3], int64_t side[3]) {
  const double D = reach * (1.0 + 1e-6);
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

template <int DIM, class T, bool FILL>
__global__ void __launch_bounds__(64) k_assemble(AsmParams P) {
  __shared__ int32_t s_key[kCap];
  __shared__ double s_val[kCap];
  __shared__ int32_t s_first[kCap];
  __shared__ int32_t s_pb[FILL ? kCap : 1];
  // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, each
  // with its own L2; give XCD j the j-th contiguous chunk of cells so that
  // neighbouring cells, which read the same hash buckets, share an L2
  const int64_t chunk = (P.n_cells + kXcds - 1) / kXcds;
  const int64_t K = (int64_t)(blockIdx.x % kXcds) * chunk + blockIdx.x / kXcds;
  if (K >= P.n_cells) return;
  const int lane = threadIdx.x;
  const int nbpc = P.nbpc;
  const int spb = kWave / nbpc;         // lanes per tracked ball
  const int s = lane / spb;
  const int slot = lane % spb;
  const int64_t b = K * nbpc + s;
  const int64_t nb = P.n_balls;

  T p[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) p[a] = (T)P.tracked[a * nb + b];
  const T ra = (T)P.r_hat[b];
  // buckets that can hold a centre within ra + r_max of p (range widened by
  // a relative 1e-6 so that binary32 rounding of the predicate cannot reach
  // past it; the predicate alone decides)
  int64_t blo[3] = {0, 0, 0}, side[3] = {1, 1, 1};
  search_range<DIM>(P, p, (double)ra + P.rmax, blo, side);
  const int nq = (int)(side[0] * side[1] * side[2]);
  const double mass = P.rho[K] * P.phi[K] * P.bvol[b];   // rho_K phi_K |B_{K,s}|

  // pass 1: number of overlaps and S = sum omega for this lane's buckets
  int cnt = 0;
  double S = 0.0;
  for (int q = slot; q < nq; q += spb) {
    const int64_t bc0 = blo[0] + q % side[0];
    const int64_t bc1 = blo[1] + (q / side[0]) % side[1];
    const int64_t bc2 = DIM == 3 ? blo[2] + q / (side[0] * side[1]) : 0;
    const int64_t bucket = bc0 + P.nbk[0] * (bc1 + P.nbk[1] * bc2);
    const int32_t lo = P.bucket_start[bucket], hi = P.bucket_start[bucket + 1];
    for (int32_t e = lo; e < hi; ++e) {
      T c[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < DIM; ++a)
        c[a] = sizeof(T) == 8 ? (T)P.bk_cen[a * nb + e] : (T)P.bk_cen32[a * nb + e];
      const T rb = (T)P.bk_rad[e];
      T d2;
      if (!overlap<DIM, T>(p, c, ra + rb, d2)) continue;
      const int64_t M = P.bk_ball[e] / nbpc;
      const double om = P.rho[M] * P.phi[M] * (double)lens<DIM, T>(ra, rb, sqrt(d2));
      S += om;
      ++cnt;
    }
  }
  // S of the ball: fixed-order butterfly over the lanes of its group
  for (int o = spb / 2; o > 0; o >>= 1) S += __shfl_xor(S, o, kWave);
  if (slot == 0 && !(S > 0.0)) atomicMin(&P.flags[0], (int32_t)b);
  const double share = S > 0.0 ? mass / S : 0.0;

  // compaction offsets (lane order) and total
  const int incl = wave_incl_scan_i(cnt);
  const int H = __shfl(incl, kWave - 1, kWave);
  int off = incl - cnt;
  if (H > kCap) {
    if (lane == 0) atomicMax(&P.flags[1], H);
    return;
  }
  // pass 2: the same overlaps, written in order
  for (int q = slot; q < nq; q += spb) {
    const int64_t bc0 = blo[0] + q % side[0];
    const int64_t bc1 = blo[1] + (q / side[0]) % side[1];
    const int64_t bc2 = DIM == 3 ? blo[2] + q / (side[0] * side[1]) : 0;
    const int64_t bucket = bc0 + P.nbk[0] * (bc1 + P.nbk[1] * bc2);
    const int32_t lo = P.bucket_start[bucket], hi = P.bucket_start[bucket + 1];
    for (int32_t e = lo; e < hi; ++e) {
      T c[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < DIM; ++a)
        c[a] = sizeof(T) == 8 ? (T)P.bk_cen[a * nb + e] : (T)P.bk_cen32[a * nb + e];
      const T rb = (T)P.bk_rad[e];
      T d2;
      if (!overlap<DIM, T>(p, c, ra + rb, d2)) continue;
      const int32_t rb_id = P.bk_ball[e];
      const int32_t M = rb_id / nbpc;
      const double om = P.rho[M] * P.phi[M] * (double)lens<DIM, T>(ra, rb, sqrt(d2));
      s_key[off] = M;
      s_val[off] = share * om;
      if (FILL) s_pb[off] = rb_id;
      ++off;
    }
  }
  __syncthreads();
  // first occurrence of every residing cell
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
      P.row_cnt[K] = u;
      P.pair_cnt[K] = H;
    }
    return;
  }
  const int32_t base = P.row_ptr[K];
  for (int e = lane; e < H; e += kWave) {
    if (!s_first[e]) continue;
    const int32_t k = s_key[e];
    int rank = 0;
    double v = 0.0;
    for (int j = 0; j < H; ++j) {
      const int32_t kj = s_key[j];
      if (s_first[j] && kj < k) ++rank;
      if (kj == k) v += s_val[j];
    }
    P.col[base + rank] = k;
    P.val[base + rank] = v;
  }
  if (P.pair_a) {
    const int32_t pb = P.pair_ptr[K];
    for (int e = lane; e < H; e += kWave) {
      // tracked ball of entry e: the group whose compacted range holds e
      P.pair_a[pb + e] = -1;
      P.pair_b[pb + e] = s_pb[e];
    }
  }
}

// The tracked ball of each pair entry: recomputed from the per-ball counts
// written by a small kernel (entries are grouped by ball, in ball order).
__global__ void k_pair_balls(const int32_t* __restrict__ pair_ptr, int64_t n_cells, int nbpc,
                             const int32_t* __restrict__ ball_cnt,
                             int32_t* __restrict__ pair_a) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= n_cells) return;
  int32_t e = pair_ptr[K];
  for (int s = 0; s < nbpc; ++s) {
    const int64_t b = K * nbpc + s;
    for (int32_t i = 0; i < ball_cnt[b]; ++i) pair_a[e++] = (int32_t)b;
  }
}

// Per-ball overlap counts (for the pair export), one thread per ball.
template <int DIM, class T>
__global__ void k_ball_counts(AsmParams P, int32_t* __restrict__ ball_cnt) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= P.n_balls) return;
  const int64_t nb = P.n_balls;
  T p[3] = {0, 0, 0};
  for (int a = 0; a < DIM; ++a) p[a] = (T)P.tracked[a * nb + b];
  const T ra = (T)P.r_hat[b];
  int64_t blo[3] = {0, 0, 0}, side[3] = {1, 1, 1};
  search_range<DIM>(P, p, (double)ra + P.rmax, blo, side);
  const int nq = (int)(side[0] * side[1] * side[2]);
  int cnt = 0;
  for (int q = 0; q < nq; ++q) {
    const int64_t bc0 = blo[0] + q % side[0];
    const int64_t bc1 = blo[1] + (q / side[0]) % side[1];
    const int64_t bc2 = DIM == 3 ? blo[2] + q / (side[0] * side[1]) : 0;
    const int64_t bucket = bc0 + P.nbk[0] * (bc1 + P.nbk[1] * bc2);
    for (int32_t e = P.bucket_start[bucket]; e < P.bucket_start[bucket + 1]; ++e) {
      T c[3] = {0, 0, 0};
      for (int a = 0; a < DIM; ++a)
        c[a] = sizeof(T) == 8 ? (T)P.bk_cen[a * nb + e] : (T)P.bk_cen32[a * nb + e];
      T d2;
      if (overlap<DIM, T>(p, c, ra + (T)P.bk_rad[e], d2)) ++cnt;
    }
  }
  ball_cnt[b] = cnt;
}

template <int DIM, class T>
static void launch_assemble(AsmParams& P, bool fill, hipStream_t s) {
  if (fill)
    {
      ::bchar::ProfScope ps_("k_assemble", s);
      k_assemble<DIM, T, true><<<(unsigned)xcd_grid(P.n_cells), 64, 0, s>>>(P);
    }
  else
    {
      ::bchar::ProfScope ps_("k_assemble", s);
      k_assemble<DIM, T, false><<<(unsigned)xcd_grid(P.n_cells), 64, 0, s>>>(P);
    }
  BCHAR_HIP(hipGetLastError());
}

static void dispatch_assemble(int dim, int precision, AsmParams& P, bool fill, hipStream_t s) {
  if (dim == 2) {
    if (precision == BCHAR_FP64)
      launch_assemble<2, double>(P, fill, s);
    else
      launch_assemble<2, float>(P, fill, s);
  } else {
    if (precision == BCHAR_FP64)
      launch_assemble<3, double>(P, fill, s);
    else
      launch_assemble<3, float>(P, fill, s);
  }
}

bchar_status assemble_v(bchar_mesh_s* m, const double* tracked, const double* r_hat,
                        int precision, bool keep_pairs, bchar_transfer_s* t,
                        int64_t* first_void, hipStream_t s) {
  Arena& ws = t->ws;
  const int64_t nc = m->n_cells;
  BCHAR_REQUIRE(kWave % m->nbpc == 0, BCHAR_E_UNSUPPORTED, "balls per cell must divide 64");
  AsmParams P{};
  P.n_cells = nc;
  P.n_balls = m->n_balls;
  P.nbpc = m->nbpc;
  for (int a = 0; a < 3; ++a) {
    P.nbk[a] = m->nbk[a];
    P.org[a] = m->box_lo[a];
  }
  P.inv_hs = 1.0 / m->hs;
  P.hs = m->hs;
  P.rmax = m->rmax;
  P.rho = m->rho.as<double>();
  P.bvol = m->bvol.as<double>();
  P.phi = m->phi.as<double>();
  P.tracked = tracked;
  P.r_hat = r_hat;
  P.bucket_start = m->bucket_start.as<int32_t>();
  P.bk_cen = m->bk_cen.as<double>();
  P.bk_cen32 = m->bk_cen32.as<float>();
  P.bk_ball = m->bk_ball.as<int32_t>();
  P.bk_rad = m->bk_rad.as<double>();
  P.row_cnt = ws.get<int32_t>(nc + 1);
  P.pair_cnt = ws.get<int32_t>(nc + 1);
  P.flags = ws.get<int32_t>(2);
  int32_t hflags[2] = {INT32_MAX, 0};
  BCHAR_HIP(hipMemcpyAsync(P.flags, hflags, sizeof(hflags), hipMemcpyHostToDevice, s));

  dispatch_assemble(m->dim, precision, P, false, s);
  BCHAR_HIP(hipMemcpyAsync(hflags, P.flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
  BCHAR_HIP(hipStreamSynchronize(s));
  if (hflags[1] > 0)
    throw Error{BCHAR_E_UNSUPPORTED, "a tracked cell overlaps " + std::to_string(hflags[1]) +
                                         " residing balls (more than " +
                                         std::to_string(kCap) + ")"};
  if (hflags[0] != INT32_MAX) {
    *first_void = hflags[0];
    return BCHAR_E_VOID_ROW;
  }
  t->row_ptr.reserve(sizeof(int32_t) * (nc + 1));
  int32_t* row_ptr = t->row_ptr.as<int32_t>();
  const int64_t nnz = exclusive_scan_i32(P.row_cnt, row_ptr, nc, ws, s);
  int32_t* pair_ptr = ws.get<int32_t>(nc + 1);
  const int64_t npairs = exclusive_scan_i32(P.pair_cnt, pair_ptr, nc, ws, s);
  t->nnz = nnz;
  t->n_pairs = npairs;
  t->col.reserve(sizeof(int32_t) * (nnz + 1));
  t->V.reserve(sizeof(double) * (nnz + 1));
  P.row_ptr = row_ptr;
  P.pair_ptr = pair_ptr;
  P.col = t->col.as<int32_t>();
  P.val = t->V.as<double>();
  P.pair_a = nullptr;
  P.pair_b = nullptr;
  if (keep_pairs) {
    t->pair_a.reserve(sizeof(int32_t) * (npairs + 1));
    t->pair_b.reserve(sizeof(int32_t) * (npairs + 1));
    P.pair_a = t->pair_a.as<int32_t>();
    P.pair_b = t->pair_b.as<int32_t>();
  }
  dispatch_assemble(m->dim, precision, P, true, s);
  if (keep_pairs) {
    int32_t* ball_cnt = ws.get<int32_t>(m->n_balls);
    if (m->dim == 2) {
      if (precision == BCHAR_FP64)
        {
          ::bchar::ProfScope ps_("k_ball_counts", s);
          k_ball_counts<2, double><<<blocks_for(m->n_balls, 128), 128, 0, s>>>(P, ball_cnt);
        }
      else
        {
          ::bchar::ProfScope ps_("k_ball_counts", s);
          k_ball_counts<2, float><<<blocks_for(m->n_balls, 128), 128, 0, s>>>(P, ball_cnt);
        }
    } else {
      if (precision == BCHAR_FP64)
        {
          ::bchar::ProfScope ps_("k_ball_counts", s);
          k_ball_counts<3, double><<<blocks_for(m->n_balls, 128), 128, 0, s>>>(P, ball_cnt);
        }
      else
        {
          ::bchar::ProfScope ps_("k_ball_counts", s);
          k_ball_counts<3, float><<<blocks_for(m->n_balls, 128), 128, 0, s>>>(P, ball_cnt);
        }
    }
    BCHAR_HIP(hipGetLastError());
    {
      ::bchar::ProfScope ps_("k_pair_balls", s);
      k_pair_balls<<<blocks_for(nc, 128), 128, 0, s>>>(pair_ptr, nc, m->nbpc, ball_cnt,
                                                       P.pair_a);
    }
    BCHAR_HIP(hipGetLastError());
  }
  return BCHAR_OK;
}

}  // namespace bchar
