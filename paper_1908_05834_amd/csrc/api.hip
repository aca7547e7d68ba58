// The extern "C" entry points declared in include/bchar.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace bchar {
const char* last_error_cstr();
}

using bchar::Error;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int64_t kMassIntoMaxCells = ((int64_t)1 << 31) - 1;

// ---- simplicial meshes (host side, at creation)

// d! times the signed measure of (a, b, c[, d]), the same expansion and
// operation order as the device's point location
double orient_host(int dim, const double* a, const double* b, const double* c,
                   const double* d) {
#pragma clang fp contract(off)
  double e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0}, e3[3] = {0, 0, 0};
  for (int k = 0; k < dim; ++k) {
    e1[k] = b[k] - a[k];
    e2[k] = c[k] - a[k];
    if (dim == 3) e3[k] = d[k] - a[k];
  }
  if (dim == 2) return e1[0] * e2[1] - e1[1] * e2[0];
  const double m0 = e2[1] * e3[2] - e2[2] * e3[1];
  const double m1 = e2[0] * e3[2] - e2[2] * e3[0];
  const double m2 = e2[0] * e3[1] - e2[1] * e3[0];
  return (e1[0] * m0 - e1[1] * m1) + e1[2] * m2;
}

// y - c^3 for c near y^(1/3), in double-double: c^2 = p + q exactly, c^3 =
// p c + q c with each product split exactly by fma, the leading difference
// y - p c exact by Sterbenz (p c is within a few units of y).
static double cube_residual(double y, double c) {
#pragma clang fp contract(off)
  const double p = c * c, q = std::fma(c, c, -p);
  const double a = p * c, ae = std::fma(p, c, -a);
  const double b = q * c, be = std::fma(q, c, -b);
  return (((y - a) - ae) - b) - be;
}

// The binary64 number nearest to the real cube root of y > 0: the C
// library's cbrt (a few units in the last place off) corrected by one
// Newton step on the double-double residual, then among that and its two
// neighbours on each side the one whose cube is closest to y; this
// decides every case except a tie within ~1e-16 of a rounding midpoint.
double cbrt_nearest(double y) {
#pragma clang fp contract(off)
  const double r0 = std::cbrt(y);
  double c = r0 + cube_residual(y, r0) / (3.0 * r0 * r0);
  const double r1 = c;
  for (int i = 0; i < 2; ++i) c = std::nextafter(c, 0.0);
  double best = r1, best_err = HUGE_VAL;
  for (int k = 0; k < 5; ++k, c = std::nextafter(c, HUGE_VAL)) {
    const double err = std::fabs(cube_residual(y, c));
    if (err < best_err) {
      best = c;
      best_err = err;
    }
  }
  return best;
}

struct SimplexHost {
  int dim = 0;
  int64_t nv = 0, nc = 0;
  std::vector<double> vtx;       // SoA, dim * nv
  std::vector<int32_t> cells;    // (dim + 1) * nc
  std::vector<double> vol, cen, rad, bvol, rho;   // cen SoA dim * nc
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  double rmax = 0;
};

// |K| = |orient| / dim!, centroid (((v0 + v1) + v2) (+ v3)) / (dim + 1), the
// ball with |B| = |K| (radius sqrt(|K| / pi) or the nearest cbrt(3 |K| / (4 pi))),
// rho_K = |K| / |B|, and the domain box
void simplex_geometry(const bchar_mesh_desc* d, SimplexHost& h) {
#pragma clang fp contract(off)
  const int dim = d->dim;
  h.dim = dim;
  h.nv = d->n_vertices;
  h.nc = d->n_simplices;
  h.vtx.resize((size_t)dim * h.nv);
  for (int a = 0; a < 3; ++a) {
    h.lo[a] = a < dim ? HUGE_VAL : 0.0;
    h.hi[a] = a < dim ? -HUGE_VAL : 0.0;
  }
  for (int64_t v = 0; v < h.nv; ++v)
    for (int a = 0; a < dim; ++a) {
      const double x = d->vertices[v * dim + a];
      BCHAR_REQUIRE(std::isfinite(x), BCHAR_E_INVALID_ARG, "vertex coordinates must be finite");
      h.vtx[(size_t)a * h.nv + v] = x;
      h.lo[a] = std::min(h.lo[a], x);
      h.hi[a] = std::max(h.hi[a], x);
    }
  h.cells.assign(d->cells, d->cells + (size_t)(dim + 1) * h.nc);
  h.vol.resize(h.nc);
  h.cen.resize((size_t)dim * h.nc);
  h.rad.resize(h.nc);
  h.bvol.resize(h.nc);
  h.rho.resize(h.nc);
  for (int64_t K = 0; K < h.nc; ++K) {
    double p[4][3] = {{0}};
    for (int i = 0; i <= dim; ++i) {
      const int32_t q = h.cells[(size_t)K * (dim + 1) + i];
      BCHAR_REQUIRE(q >= 0 && q < h.nv, BCHAR_E_INVALID_ARG, "cell vertex id out of range");
      for (int a = 0; a < dim; ++a) p[i][a] = h.vtx[(size_t)a * h.nv + q];
    }
    const double o = orient_host(dim, p[0], p[1], p[2], p[dim == 3 ? 3 : 2]);
    const double v = std::fabs(o) / (dim == 2 ? 2.0 : 6.0);
    BCHAR_REQUIRE(v > 0, BCHAR_E_INVALID_ARG, "degenerate simplex");
    h.vol[K] = v;
    for (int a = 0; a < dim; ++a) {
      double acc = p[0][a] + p[1][a];
      for (int i = 2; i <= dim; ++i) acc = acc + p[i][a];
      h.cen[(size_t)a * h.nc + K] = acc / (double)(dim + 1);
    }
    const double r =
        dim == 2 ? std::sqrt(v / kPi) : cbrt_nearest(3.0 * v / (4.0 * kPi));
    h.rad[K] = r;
    h.bvol[K] = dim == 2 ? kPi * r * r : 4.0 / 3.0 * kPi * r * r * r;
    h.rho[K] = v / h.bvol[K];
    h.rmax = std::max(h.rmax, r);
  }
}

// Several disjoint balls per simplex (layout PACKED): the inscribed ball
// (incentre sum_i w_i v_i / sum_i w_i, w_i the measure of the facet
// opposite v_i; radius dim |K| / sum_i w_i), then for every vertex the ball
// tangent to the facets through it and to the inscribed ball (centre
// v_i + t (I - v_i), radius t r, t = (L - r) / (L + r), L = |v_i - I|),
// every radius times kPackShrink; a cell whose balls still overlap keeps
// the inscribed ball alone.  Output in the CUSTOM format (ball-major
// centre then radius; the cell of every ball).
constexpr double kPackShrink = 0.875;

void packed_simplex_balls(const SimplexHost& h, std::vector<double>& balls,
                          std::vector<int32_t>& ball_cell) {
#pragma clang fp contract(off)
  const int dim = h.dim;
  const int nb = dim + 2;
  balls.clear();
  ball_cell.clear();
  balls.reserve((size_t)h.nc * nb * (dim + 1));
  ball_cell.reserve((size_t)h.nc * nb);
  for (int64_t K = 0; K < h.nc; ++K) {
    double p[4][3] = {{0}};
    for (int i = 0; i <= dim; ++i) {
      const int32_t q = h.cells[(size_t)K * (dim + 1) + i];
      for (int a = 0; a < dim; ++a) p[i][a] = h.vtx[(size_t)a * h.nv + q];
    }
    double w[4] = {0, 0, 0, 0};
    for (int i = 0; i <= dim; ++i) {
      int o[3], k = 0;
      for (int j = 0; j <= dim; ++j)
        if (j != i) o[k++] = j;
      if (dim == 2) {
        const double e0 = p[o[1]][0] - p[o[0]][0], e1 = p[o[1]][1] - p[o[0]][1];
        w[i] = std::sqrt(e0 * e0 + e1 * e1);
      } else {
        double u[3], v[3];
        for (int a = 0; a < 3; ++a) {
          u[a] = p[o[1]][a] - p[o[0]][a];
          v[a] = p[o[2]][a] - p[o[0]][a];
        }
        const double c0 = u[1] * v[2] - u[2] * v[1];
        const double c1 = u[2] * v[0] - u[0] * v[2];
        const double c2 = u[0] * v[1] - u[1] * v[0];
        w[i] = std::sqrt((c0 * c0 + c1 * c1) + c2 * c2) / 2.0;
      }
    }
    double W = w[0] + w[1];
    for (int i = 2; i <= dim; ++i) W = W + w[i];
    double inc[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
      double acc = w[0] * p[0][a] + w[1] * p[1][a];
      for (int i = 2; i <= dim; ++i) acc = acc + w[i] * p[i][a];
      inc[a] = acc / W;
    }
    const double r = ((double)dim * h.vol[K]) / W;
    double c[5][3] = {{0}}, rad[5] = {0, 0, 0, 0, 0};
    for (int a = 0; a < dim; ++a) c[0][a] = inc[a];
    rad[0] = kPackShrink * r;
    for (int i = 0; i <= dim; ++i) {
      double d[3];
      for (int a = 0; a < dim; ++a) d[a] = p[i][a] - inc[a];
      double L2 = d[0] * d[0];
      for (int a = 1; a < dim; ++a) L2 = L2 + d[a] * d[a];
      const double L = std::sqrt(L2);
      const double t = (L - r) / (L + r);
      for (int a = 0; a < dim; ++a) c[1 + i][a] = p[i][a] + t * (inc[a] - p[i][a]);
      rad[1 + i] = kPackShrink * (t * r);
    }
    bool ok = true;
    for (int a = 0; a < nb; ++a)
      for (int b = a + 1; b < nb; ++b) {
        double d2 = 0;
        for (int k = 0; k < dim; ++k) {
          const double dk = c[a][k] - c[b][k];
          d2 = k == 0 ? dk * dk : d2 + dk * dk;
        }
        ok = ok && std::sqrt(d2) >= rad[a] + rad[b];
      }
    const int take = ok ? nb : 1;
    for (int q = 0; q < take; ++q) {
      for (int a = 0; a < dim; ++a) balls.push_back(c[q][a]);
      balls.push_back(rad[q]);
      ball_cell.push_back((int32_t)K);
    }
  }
}

// Device copies, and (when phi varies, so that tracking needs it) the
// uniform grid of side (|box| / n_cells)^(1/dim) listing, per grid cell
// and in ascending order, the cells whose bounding box meets it.
void simplex_upload(bchar_mesh_s* m, const SimplexHost& h, const std::vector<double>& b,
                    bool centroid_balls, hipStream_t s) {
  const int dim = h.dim;
  auto up = [&](bchar::DBuf& buf, const void* src, size_t bytes) {
    buf.reserve(bytes);
    BCHAR_HIP(hipMemcpyAsync(buf.p, src, bytes, hipMemcpyHostToDevice, s));
  };
  up(m->cell_cen, h.cen.data(), sizeof(double) * h.cen.size());
  if (centroid_balls) {
    std::vector<float> cen32(h.cen.size());
    for (size_t i = 0; i < h.cen.size(); ++i) cen32[i] = (float)h.cen[i];
    up(m->cen, h.cen.data(), sizeof(double) * h.cen.size());
    up(m->cen32, cen32.data(), sizeof(float) * cen32.size());
    up(m->rad, h.rad.data(), sizeof(double) * h.nc);
    up(m->bvol, h.bvol.data(), sizeof(double) * h.nc);
    up(m->rho, h.rho.data(), sizeof(double) * h.nc);
    m->rmax = h.rmax;
  }
  up(m->b, b.data(), sizeof(double) * h.nc);
  up(m->vtx, h.vtx.data(), sizeof(double) * h.vtx.size());
  up(m->cells, h.cells.data(), sizeof(int32_t) * h.cells.size());
  m->n_vertices = h.nv;
  std::vector<int32_t> start, list;
  double side = 1.0;
  int64_t nb[3] = {1, 1, 1};
  if (!m->phi_const) {
    double boxvol = 1.0;
    for (int a = 0; a < dim; ++a) boxvol *= std::max(h.hi[a] - h.lo[a], 1e-300);
    side = std::pow(boxvol / (double)h.nc, 1.0 / dim);
    int64_t ng = 1;
    for (int a = 0; a < dim; ++a) {
      nb[a] = std::max<int64_t>(1, (int64_t)std::ceil((h.hi[a] - h.lo[a]) / side));
      ng *= nb[a];
    }
    BCHAR_REQUIRE(ng < ((int64_t)1 << 31), BCHAR_E_UNSUPPORTED, "location grid too large");
    const double inv = 1.0 / side;
    auto range = [&](int64_t K, int64_t lo_i[3], int64_t hi_i[3]) {
      for (int a = 0; a < 3; ++a) {
        lo_i[a] = 0;
        hi_i[a] = 0;
      }
      for (int a = 0; a < dim; ++a) {
        double lo = HUGE_VAL, hi = -HUGE_VAL;
        for (int i = 0; i <= dim; ++i) {
          const double x = h.vtx[(size_t)a * h.nv + h.cells[(size_t)K * (dim + 1) + i]];
          lo = std::min(lo, x);
          hi = std::max(hi, x);
        }
        int64_t l = (int64_t)std::floor((lo - h.lo[a]) * inv);
        int64_t u = (int64_t)std::floor((hi - h.lo[a]) * inv);
        lo_i[a] = std::min(std::max<int64_t>(l, 0), nb[a] - 1);
        hi_i[a] = std::min(std::max<int64_t>(u, 0), nb[a] - 1);
      }
    };
    std::vector<int64_t> cnt(ng + 1, 0);
    for (int64_t K = 0; K < h.nc; ++K) {
      int64_t l[3], u[3];
      range(K, l, u);
      for (int64_t k = l[2]; k <= u[2]; ++k)
        for (int64_t j = l[1]; j <= u[1]; ++j)
          for (int64_t i = l[0]; i <= u[0]; ++i) ++cnt[i + nb[0] * (j + nb[1] * k) + 1];
    }
    for (int64_t g = 0; g < ng; ++g) cnt[g + 1] += cnt[g];
    BCHAR_REQUIRE(cnt[ng] < ((int64_t)1 << 31), BCHAR_E_UNSUPPORTED, "location lists too long");
    start.assign(cnt.begin(), cnt.end());
    list.resize(cnt[ng]);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t K = 0; K < h.nc; ++K) {
      int64_t l[3], u[3];
      range(K, l, u);
      for (int64_t k = l[2]; k <= u[2]; ++k)
        for (int64_t j = l[1]; j <= u[1]; ++j)
          for (int64_t i = l[0]; i <= u[0]; ++i)
            list[pos[i + nb[0] * (j + nb[1] * k)]++] = (int32_t)K;
    }
  } else {
    start.assign(2, 0);
    list.assign(1, 0);
  }
  m->pl_inv = 1.0 / side;
  for (int a = 0; a < 3; ++a) m->pl_nb[a] = nb[a];
  up(m->pl_start, start.data(), sizeof(int32_t) * start.size());
  up(m->pl_list, list.data(), sizeof(int32_t) * list.size());
  BCHAR_HIP(hipStreamSynchronize(s));
}

// The caller's balls (layout CUSTOM, Sec. 3: any points C_{K,s} with radii
// r_{K,s}, a cell's balls consecutive): ball measures, rho_K = |K| / sum_s
// |B_{K,s}| (eq. def:porous.density, the measures summed in ball order),
// the first ball of every cell, and tiles of whole cells with at most 256
// balls each for the assembly.
void custom_layout(bchar_mesh_s* m, int64_t nb, const double* balls, const int32_t* ball_cell,
                   const std::vector<double>& kvol, hipStream_t s) {
#pragma clang fp contract(off)
  const int dim = m->dim;
  const int64_t nc = m->n_cells;
  BCHAR_REQUIRE(nb >= nc && nb < ((int64_t)1 << 31) - 1, BCHAR_E_INVALID_ARG,
                "CUSTOM layout: n_balls must be >= the number of cells and < 2^31");
  BCHAR_REQUIRE(balls != nullptr && ball_cell != nullptr, BCHAR_E_INVALID_ARG,
                "CUSTOM layout: balls or ball_cell is NULL");
  std::vector<int32_t> ptr(nc + 1, 0);
  std::vector<double> cen((size_t)dim * nb), rad(nb), bvol(nb), rho(nc);
  std::vector<float> cen32((size_t)dim * nb);
  double rmax = 0;
  bool uniform = true;
  for (int64_t i = 0; i < nb; ++i) {
    const int32_t K = ball_cell[i];
    BCHAR_REQUIRE(K >= 0 && K < nc, BCHAR_E_INVALID_ARG, "CUSTOM layout: ball_cell out of range");
    BCHAR_REQUIRE(i == 0 ? K == 0 : (K == ball_cell[i - 1] || K == ball_cell[i - 1] + 1),
                  BCHAR_E_INVALID_ARG,
                  "CUSTOM layout: ball_cell must start at 0 and step by 0 or 1 (every cell "
                  "owns at least one ball, a cell's balls consecutive)");
    ++ptr[K + 1];
    for (int a = 0; a < dim; ++a) {
      const double x = balls[i * (dim + 1) + a];
      BCHAR_REQUIRE(std::isfinite(x), BCHAR_E_INVALID_ARG, "CUSTOM layout: centre not finite");
      cen[(size_t)a * nb + i] = x;
      cen32[(size_t)a * nb + i] = (float)x;
    }
    const double r = balls[i * (dim + 1) + dim];
    BCHAR_REQUIRE(r > 0 && std::isfinite(r), BCHAR_E_INVALID_ARG,
                  "CUSTOM layout: radius must be finite and > 0");
    rad[i] = r;
    bvol[i] = dim == 2 ? kPi * r * r : 4.0 / 3.0 * kPi * r * r * r;
    rmax = std::max(rmax, r);
    uniform = uniform && r == rad[0];
  }
  BCHAR_REQUIRE(ball_cell[nb - 1] == nc - 1, BCHAR_E_INVALID_ARG,
                "CUSTOM layout: every cell needs at least one ball");
  for (int64_t K = 0; K < nc; ++K) {
    BCHAR_REQUIRE(ptr[K + 1] <= 256, BCHAR_E_UNSUPPORTED,
                  "CUSTOM layout: more than 256 balls in one cell");
    ptr[K + 1] += ptr[K];
  }
  for (int64_t K = 0; K < nc; ++K) {
    double sum = 0.0;
    for (int32_t i = ptr[K]; i < ptr[K + 1]; ++i) sum = sum + bvol[i];
    rho[K] = kvol[K] / sum;
  }
  std::vector<int32_t> tiles(1, 0);
  for (int64_t K = 0; K < nc;) {
    int64_t e = K;
    while (e < nc && ptr[e + 1] - ptr[K] <= 256) ++e;
    tiles.push_back((int32_t)e);
    K = e;
  }
  auto up = [&](bchar::DBuf& buf, const void* src, size_t bytes) {
    buf.reserve(bytes);
    BCHAR_HIP(hipMemcpyAsync(buf.p, src, bytes, hipMemcpyHostToDevice, s));
  };
  up(m->cen, cen.data(), sizeof(double) * cen.size());
  up(m->cen32, cen32.data(), sizeof(float) * cen32.size());
  up(m->rad, rad.data(), sizeof(double) * nb);
  up(m->bvol, bvol.data(), sizeof(double) * nb);
  up(m->rho, rho.data(), sizeof(double) * nc);
  up(m->ball_ptr, ptr.data(), sizeof(int32_t) * (nc + 1));
  up(m->ball_cell, ball_cell, sizeof(int32_t) * nb);
  up(m->tile_cell, tiles.data(), sizeof(int32_t) * tiles.size());
  BCHAR_HIP(hipStreamSynchronize(s));
  m->n_tiles = (int64_t)tiles.size() - 1;
  m->nbpc = 0;
  m->n_balls = nb;
  m->rmax = rmax;
  m->r_uniform = uniform;
  m->r0 = rad[0];
}

template <class F>
bchar_status guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    bchar::set_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    bchar::set_error("host allocation failed");
    return BCHAR_E_OUT_OF_MEMORY;
  } catch (...) {
    bchar::set_error("unexpected exception");
    return BCHAR_E_DEVICE;
  }
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

void opts_or_default(const bchar_opts* in, bchar_opts& o) {
  if (in)
    o = *in;
  else
    bchar_opts_default(&o);
}

void validate_opts(const bchar_opts& o) {
  BCHAR_REQUIRE(o.precision == BCHAR_FP64 || o.precision == BCHAR_FP32_VOLUME ||
                    o.precision == BCHAR_FP32_LENS,
                BCHAR_E_INVALID_ARG, "opts.precision");
  BCHAR_REQUIRE(o.n_sweeps >= 0 && o.n_sweeps <= 100000, BCHAR_E_INVALID_ARG, "opts.n_sweeps");
  BCHAR_REQUIRE(o.rk_substeps >= 1 && o.rk_substeps <= 4096, BCHAR_E_INVALID_ARG,
                "opts.rk_substeps");
  BCHAR_REQUIRE(o.box_policy == BCHAR_BOX_PAPER_THEN_RELAX || o.box_policy == BCHAR_BOX_STRICT,
                BCHAR_E_INVALID_ARG, "opts.box_policy");
  BCHAR_REQUIRE(o.stop_after >= BCHAR_STAGE_PAIRS && o.stop_after <= BCHAR_STAGE_ALL,
                BCHAR_E_INVALID_ARG, "opts.stop_after");
  BCHAR_REQUIRE(o.qp_tol > 0 && std::isfinite(o.qp_tol), BCHAR_E_INVALID_ARG, "opts.qp_tol");
  BCHAR_REQUIRE(o.qp_max_newton >= 1 && o.qp_max_cg >= 1, BCHAR_E_INVALID_ARG,
                "opts.qp_max_newton / qp_max_cg");
  BCHAR_REQUIRE(o.max_halvings >= 0 && o.max_halvings <= 20, BCHAR_E_INVALID_ARG,
                "opts.max_halvings");
  BCHAR_REQUIRE(o.z_fuse_max_cells >= 0, BCHAR_E_INVALID_ARG, "opts.z_fuse_max_cells");
  BCHAR_REQUIRE(o.divergence == BCHAR_DIV_FREE || o.divergence == BCHAR_DIV_GENERAL,
                BCHAR_E_INVALID_ARG, "opts.divergence");
  BCHAR_REQUIRE(o.tile_aspect >= -4 && o.tile_aspect <= 4, BCHAR_E_INVALID_ARG,
                "opts.tile_aspect");
}

void validate_velocity(const bchar_mesh_s* m, const bchar_velocity* u) {
  BCHAR_REQUIRE(u != nullptr, BCHAR_E_INVALID_ARG, "velocity is NULL");
  for (int a = 0; a < m->dim; ++a) {
    BCHAR_REQUIRE(u->m[a] >= 2, BCHAR_E_INVALID_ARG, "velocity lattice needs >= 2 nodes per axis");
    BCHAR_REQUIRE(u->spacing[a] > 0 && std::isfinite(u->spacing[a]) &&
                      std::isfinite(u->origin[a]),
                  BCHAR_E_INVALID_ARG, "velocity lattice spacing/origin");
    BCHAR_REQUIRE(u->u[a] != nullptr, BCHAR_E_INVALID_ARG, "velocity component is NULL");
  }
  int64_t nn = 1;
  for (int a = 0; a < m->dim; ++a) nn *= u->m[a];
  BCHAR_REQUIRE(nn < ((int64_t)1 << 31), BCHAR_E_UNSUPPORTED, "velocity lattice too large");
}

// Everything after the tracked centres are known.
bchar_status build_from_tracked(bchar_mesh_s* m, bchar_transfer_s* t, const bchar_opts& o,
                                int trace_precision, hipStream_t s, bchar_stats* stats) {
  using namespace bchar;
  Arena& ws = t->ws;
  const bool tr = trace_enabled();
  double t0 = 0;
  if (tr) {
    BCHAR_HIP(hipStreamSynchronize(s));
    t0 = wall_seconds();
  }
  bchar_stats st{};
  st.n_balls = m->n_balls;
  st.first_void = -1;
  st.trace_precision = trace_precision;
  st.row_target_scale = 1.0;
  t->stage = 0;
  int64_t first_void = -1;
  bchar_status rc = assemble_v(m, t->tracked.as<double>(), t->r_hat.as<double>(),
                               t->general ? t->lam.as<double>() : nullptr, o.precision,
                               o.keep_pairs != 0, o.lds_stage != 0, o.tile_aspect, t,
                               &first_void, s);
  st.nnz = t->nnz;
  st.n_pairs = t->n_pairs;
  st.n_void_rows = t->n_void_rows;
  if (rc != BCHAR_OK) {
    st.first_void = first_void;
    if (stats) *stats = st;
    t->stats = st;
    set_error("void row: tracked ball " + std::to_string(first_void) +
              " overlaps no residing ball");
    return rc;
  }
  t->stage = BCHAR_STAGE_V;
  if (tr) {
    BCHAR_HIP(hipStreamSynchronize(s));
    fprintf(stderr, "[bchar] V: %.3f ms (nnz %lld, pairs %lld)\n", 1e3 * (wall_seconds() - t0),
            (long long)t->nnz, (long long)t->n_pairs);
    t0 = wall_seconds();
  }
  if (o.stop_after <= BCHAR_STAGE_V) {
    BCHAR_HIP(hipStreamSynchronize(s));
    if (stats) *stats = st;
    t->stats = st;
    return BCHAR_OK;
  }
  const int64_t n = m->n_cells, nnz = t->nnz;
  t->groups = 0;
  if (t->general) {
    const TargetInfo ti = row_targets(m, t, t->lam.as<double>(), t->b_row.as<double>(), ws, s);
    st.row_target_scale = ti.scale;
    st.n_target_groups = ti.groups;
    t->groups = ti.groups;
    if (tr)
      fprintf(stderr, "[bchar] row targets: scale %.17g, %lld groups, %d rounds\n", ti.scale,
              (long long)ti.groups, ti.rounds);
  }
  Csc csc{};
  build_csc(t->row_ptr.as<int32_t>(), t->col.as<int32_t>(), n, nnz, csc, ws, s);
  t->AN.reserve(sizeof(double) * (nnz + 1));
  int64_t void_col = -1, n_void_cols = 0;
  double col_err = 0;
  // row targets: |K|_phi (eq. exactVol_traceback), or eq. volTracked's for
  // a non-solenoidal u
  const double* b_row = t->general ? t->b_row.as<double>() : m->b.as<double>();
  rc = scaling_sweeps(m, t->row_ptr.as<int32_t>(), t->col.as<int32_t>(), csc, t->V.as<double>(),
                      b_row, nnz, o.n_sweeps, t->AN.as<double>(), &void_col, &n_void_cols,
                      &col_err, ws, s);
  st.scaling_max_col_err = col_err;
  st.n_void_cols = n_void_cols;
  if (rc != BCHAR_OK) {
    st.first_void = void_col;
    if (stats) *stats = st;
    t->stats = st;
    set_error("void column: residing cell " + std::to_string(void_col) +
              " receives no tracked ball");
    return rc;
  }
  t->stage = BCHAR_STAGE_SCALING;
  if (tr) {
    fprintf(stderr, "[bchar] scaling: %.3f ms (max column error %.3e)\n",
            1e3 * (wall_seconds() - t0), col_err);
    t0 = wall_seconds();
  }
  if (o.stop_after <= BCHAR_STAGE_SCALING) {
    if (stats) *stats = st;
    t->stats = st;
    return BCHAR_OK;
  }
  t->x.reserve(sizeof(double) * (nnz + 1));
  t->A.reserve(sizeof(double) * (nnz + 1));
  t->mu.reserve(sizeof(double) * n);
  t->nu.reserve(sizeof(double) * n);
  if (t->zdual.bytes < sizeof(double) * 4 * n) {
    t->zdual.reserve(sizeof(double) * 4 * n);
    t->warm_level = -1;
  }
  if (t->warm_level < 0) t->warm_newton_skip = 0;
  QpResult qr;
  Groups grp{t->grp_lab.as<int32_t>(), t->grp_ptr.as<int32_t>(), t->grp_perm.as<int32_t>()};
  rc = solve_qp(m, t->row_ptr.as<int32_t>(), t->col.as<int32_t>(), csc, t->AN.as<double>(),
                b_row, t->groups > 1 ? &grp : nullptr, nnz, o, t->x.as<double>(),
                t->mu.as<double>(), t->nu.as<double>(), t->A.as<double>(), t->zdual.as<double>(),
                t->warm_level, t->warm_newton_skip, qr, ws, s);
  t->warm_level = rc == BCHAR_OK ? qr.level : -1;
  if (tr)
    fprintf(stderr, "[bchar] qp: %.3f ms (level %d, ipm %d, newton %d, cg %d, residual %.3e)\n",
            1e3 * (wall_seconds() - t0), qr.level, qr.ipm, qr.newton, qr.cg, qr.residual);
  st.qp_level = qr.level;
  st.qp_newton = qr.newton;
  st.qp_cg = qr.cg;
  st.qp_ipm = qr.ipm;
  st.qp_coarse_bytes = qr.coarse_bytes;
  st.qp_smooth_bytes = qr.smooth_bytes;
  st.qp_residual = qr.residual;
  st.n_at_lower = qr.at_lower;
  st.n_at_upper = qr.at_upper;
  st.qp_corrected = qr.corrected ? 1 : 0;
  if (stats) *stats = st;
  t->stats = st;
  if (rc != BCHAR_OK) {
    set_error(rc == BCHAR_E_QP_INFEASIBLE
                  ? "the box of the least-change problem admits no solution"
                  : "the least-change problem did not reach the tolerance (residual " +
                        std::to_string(qr.residual) + ")");
    return rc;
  }
  t->stage = BCHAR_STAGE_ALL;
  return BCHAR_OK;
}

bchar_status build_once(bchar_mesh_s* m, bchar_transfer_s* t, const bchar_velocity* u,
                        double dt, const bchar_opts& o, hipStream_t s, bchar_stats* stats) {
  using namespace bchar;
  BCHAR_REQUIRE(o.precision != BCHAR_FP32_VOLUME || m->phi_const, BCHAR_E_UNSUPPORTED,
                "FP32_VOLUME tracks in binary32 and needs a constant porosity; FP32_LENS "
                "tracks in binary64");
  BCHAR_REQUIRE(m->n_ghost == 0 || o.divergence == BCHAR_DIV_FREE, BCHAR_E_UNSUPPORTED,
                "ghost cells take solenoidal steps only");
  BCHAR_REQUIRE(o.precision != BCHAR_FP32_VOLUME || o.divergence == BCHAR_DIV_FREE,
                BCHAR_E_UNSUPPORTED,
                "FP32_VOLUME tracks in binary32 and needs a solenoidal u; FP32_LENS tracks in "
                "binary64");
  t->ws.reset();
  t->tracked.reserve(sizeof(double) * m->dim * m->n_balls);
  t->r_hat.reserve(sizeof(double) * m->n_balls);
  t->general = o.divergence == BCHAR_DIV_GENERAL;
  if (t->general) {
    t->lam.reserve(sizeof(double) * m->n_balls);
    t->b_row.reserve(sizeof(double) * m->n_cells);
  }
  const double t0 = trace_enabled() ? wall_seconds() : 0.0;
  trace_balls(m, *u, dt, o.rk_substeps, o.precision, t->tracked.as<double>(),
              t->r_hat.as<double>(), t->general ? t->lam.as<double>() : nullptr, t->ws, s);
  if (trace_enabled()) {
    BCHAR_HIP(hipStreamSynchronize(s));
    fprintf(stderr, "[bchar] trace: %.3f ms\n", 1e3 * (wall_seconds() - t0));
  }
  return build_from_tracked(m, t, o,
                            o.precision == BCHAR_FP32_VOLUME ? BCHAR_FP32_VOLUME : BCHAR_FP64, s,
                            stats);
}

// device memory a transfer holds (its buffers and scratch chunks)
int64_t transfer_device_bytes(const bchar_transfer_s* t) {
  const bchar::DBuf* bufs[] = {&t->row_ptr,   &t->col,       &t->V,        &t->AN,
                               &t->A,         &t->x,         &t->mu,       &t->nu,
                               &t->zdual,     &t->tracked,   &t->r_hat,    &t->lam,
                               &t->b_row,     &t->grp_lab,   &t->grp_ptr,  &t->grp_perm,
                               &t->pair_a,    &t->pair_b,    &t->stage_col, &t->stage_val,
                               &t->cscratch};
  int64_t n = 0;
  for (const auto* b : bufs) n += (int64_t)b->bytes;
  for (const auto& c : t->ws.chunks) n += (int64_t)c.bytes;
  return n;
}

// A void row or column is the method's sign that the step is too long for
// the mesh: the build is repeated with half the step (the remedy the paper
// gives), at most o.max_halvings times.
bchar_status do_build(bchar_mesh_s* m, bchar_transfer_s* t, const bchar_velocity* u, double dt,
                      const bchar_opts& o, hipStream_t s, bchar_stats* stats) {
  validate_opts(o);
  validate_velocity(m, u);
  BCHAR_REQUIRE(dt > 0 && std::isfinite(dt), BCHAR_E_INVALID_ARG, "dt must be finite and > 0");
  bchar_status rc = BCHAR_OK;
  int h = 0;
  for (;; ++h) {
    // with halve_on_level2 the least-change solve stops at level 1 (no
    // negative volumes) and reports the box infeasible, except on the last
    // allowed attempt, which may take level 2
    bchar_opts oh = o;
    if (h >= o.max_halvings) oh.halve_on_level2 = 0;
    rc = build_once(m, t, u, std::ldexp(dt, -h), oh, s, stats);
    const bool negative = rc == BCHAR_E_QP_INFEASIBLE && oh.halve_on_level2;
    if ((rc != BCHAR_E_VOID_ROW && rc != BCHAR_E_VOID_COLUMN && !negative) ||
        h >= o.max_halvings)
      break;
    if (bchar::trace_enabled())
      fprintf(stderr, "[bchar] %s: step halved to dt / %d\n", negative ? "level 2" : "void",
              1 << (h + 1));
  }
  t->substeps = 1 << h;
  t->stats.dt_halvings = h;
  t->stats.device_bytes = transfer_device_bytes(t);
  if (stats) {
    stats->dt_halvings = h;
    stats->device_bytes = t->stats.device_bytes;
  }
  return rc;
}

// The update applied t->substeps times, the last one into cout.
void apply_substeps(bchar_transfer_s* t, const double* cin, double* cout, double* tmp,
                    hipStream_t s) {
  const double* src = cin;
  for (int i = 0; i < t->substeps; ++i) {
    double* dst = ((t->substeps - 1 - i) % 2 == 0) ? cout : tmp;
    bchar::apply_transfer(t, src, dst, s);
    src = dst;
  }
}

}  // namespace

// ---------------------------------------------------------------- serving

static void transfer_free(bchar_transfer t);

struct bchar_server_s {
  struct Item {
    bchar_request req;
    int64_t bytes = 0;
    bool done = false;
    bchar_request_result res{};
  };
  int dev = 0;
  bchar_opts opts{};
  // Admission by memory: every worker keeps its transfer's buffers between
  // requests, so what counts is the memory the workers hold.  retained[w]
  // is worker w's, measured after each request and taken as at least the
  // running request's declared bytes while it runs; held is their sum.
  int64_t budget = 0, held = 0;
  std::vector<int64_t> retained;
  int running = 0;                       // requests in progress
  std::vector<hipStream_t> streams;
  std::vector<bchar_transfer_s*> transfers;   // one per worker, rebuilt per request
  std::mutex mu;
  std::condition_variable cv;            // queue, memory and completions
  std::deque<int64_t> queue;             // tickets waiting, in submission order
  std::map<int64_t, Item> items;
  int64_t next_ticket = 1;
  bool stopping = false;
  std::vector<std::thread> workers;

  // what the workers would hold if worker w took a request of `bytes`
  int64_t projected(int w, int64_t bytes) const {
    return held - retained[w] + std::max(retained[w], bytes);
  }

  void work(int w) {
    (void)hipSetDevice(dev);
    bchar_transfer_s* t = transfers[w];
    hipStream_t s = streams[w];
    for (;;) {
      int64_t ticket = 0;
      Item* it = nullptr;
      bool trim = false;
      {
        std::unique_lock<std::mutex> lk(mu);
        // the oldest request starts once the memory the workers would then
        // hold fits the budget, or alone (nothing running, no other worker
        // holding memory) when it never fits; a worker that holds memory
        // while the oldest request waits for memory gives it back
        cv.wait(lk, [&] {
          if (queue.empty()) return stopping;
          const Item& head = items[queue.front()];
          if (budget == 0 || projected(w, head.bytes) <= budget) return true;
          if (running == 0 && held == retained[w]) return true;
          if (retained[w] > 0) {
            trim = true;
            return true;
          }
          return false;
        });
        if (queue.empty()) return;
        if (!trim) {
          ticket = queue.front();
          queue.pop_front();
          it = &items[ticket];
          const int64_t r = std::max(retained[w], it->bytes);
          held += r - retained[w];
          retained[w] = r;
          ++running;
          it->res.t_start = bchar::wall_seconds();
        }
      }
      if (trim) {
        // release this worker's buffers (the next request allocates again)
        (void)hipStreamSynchronize(s);
        transfer_free(t);
        t->stage_need = t->pair_need = 0;
        {
          std::lock_guard<std::mutex> lk(mu);
          held -= retained[w];
          retained[w] = 0;
        }
        cv.notify_all();
        continue;
      }
      const bchar_request& r = it->req;
      bchar_status st = guarded([&]() -> bchar_status {
        // the transfer follows the request's mesh; a multiplier warm start
        // from another problem would be meaningless
        t->mesh = r.mesh;
        t->warm_level = -1;
        bchar_status rc = do_build(r.mesh, t, r.u, r.dt, opts, s, &it->res.stats);
        if (rc != BCHAR_OK) return rc;
        // every update is t->substeps sub-steps after void halvings
        const int k = r.steps * t->substeps;
        BCHAR_REQUIRE(k == 1 || r.c_tmp != nullptr, BCHAR_E_INVALID_ARG,
                      "request needs c_tmp (the step was halved)");
        const double* src = r.c_in;
        for (int i = 0; i < k; ++i) {
          double* dst = ((k - 1 - i) % 2 == 0) ? r.c_out : r.c_tmp;
          bchar::apply_transfer(t, src, dst, s);
          src = dst;
        }
        BCHAR_HIP(hipStreamSynchronize(s));
        return BCHAR_OK;
      });
      const int64_t now = transfer_device_bytes(t);
      {
        std::lock_guard<std::mutex> lk(mu);
        it->res.status = st;
        it->res.t_done = bchar::wall_seconds();
        it->done = true;
        held += now - retained[w];
        retained[w] = now;
        --running;
      }
      cv.notify_all();
    }
  }
};

extern "C" {

void bchar_opts_default(bchar_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = BCHAR_FP64;
  o->n_sweeps = 10;
  o->rk_substeps = 1;
  o->box_policy = BCHAR_BOX_PAPER_THEN_RELAX;
  o->stop_after = BCHAR_STAGE_ALL;
  o->qp_tol = 1e-13;
  o->qp_max_newton = 500;
  o->qp_max_cg = 400;
  o->keep_pairs = 0;
  o->warm_start = 1;
  o->cg_graphs = 1;
  o->lds_stage = 0;
  o->z_fuse_max_cells = 1 << 20;
  o->divergence = BCHAR_DIV_FREE;
  o->tile_aspect = 0;
}

const char* bchar_status_string(bchar_status s) {
  switch (s) {
    case BCHAR_OK: return "ok";
    case BCHAR_E_INVALID_ARG: return "invalid argument";
    case BCHAR_E_OUT_OF_MEMORY: return "out of memory";
    case BCHAR_E_DEVICE: return "device error";
    case BCHAR_E_VOID_ROW: return "void row";
    case BCHAR_E_VOID_COLUMN: return "void column";
    case BCHAR_E_QP_INFEASIBLE: return "least-change problem infeasible";
    case BCHAR_E_QP_NOT_CONVERGED: return "least-change problem not converged";
    case BCHAR_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* bchar_last_error(void) { return bchar::last_error_cstr(); }

bchar_status bchar_mesh_create(const bchar_mesh_desc* d, void* stream, bchar_mesh* out) {
  if (out) *out = nullptr;
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(d != nullptr && out != nullptr, BCHAR_E_INVALID_ARG, "NULL argument");
    BCHAR_REQUIRE(d->dim == 2 || d->dim == 3, BCHAR_E_INVALID_ARG, "dim must be 2 or 3");
    BCHAR_REQUIRE(d->kind == BCHAR_MESH_CARTESIAN || d->kind == BCHAR_MESH_SIMPLEX,
                  BCHAR_E_INVALID_ARG, "unknown mesh kind");
    BCHAR_REQUIRE(d->layout >= BCHAR_LAYOUT_SUBCELL && d->layout <= BCHAR_LAYOUT_PACKED,
                  BCHAR_E_INVALID_ARG, "unknown layout");
    BCHAR_REQUIRE(d->phi != nullptr, BCHAR_E_INVALID_ARG, "phi is NULL");
    BCHAR_REQUIRE(d->phi_mem == BCHAR_MEM_HOST || d->phi_mem == BCHAR_MEM_DEVICE,
                  BCHAR_E_INVALID_ARG, "phi_mem");
    BCHAR_REQUIRE(d->geom_mem == BCHAR_MEM_HOST || d->geom_mem == BCHAR_MEM_DEVICE,
                  BCHAR_E_INVALID_ARG, "geom_mem");
    hipStream_t s = as_stream(stream);
    const bool custom = d->layout == BCHAR_LAYOUT_CUSTOM;
    const bool packed = d->layout == BCHAR_LAYOUT_PACKED;
    // geometry given in device memory: host copies (creation runs on the host)
    bchar_mesh_desc dh = *d;
    std::vector<double> h_vtx, h_balls;
    std::vector<int32_t> h_cells, h_bcell;
    if (d->geom_mem == BCHAR_MEM_DEVICE) {
      auto down = [&](auto& vec, const void* src, size_t count) {
        vec.resize(count);
        if (count && src)
          BCHAR_HIP(hipMemcpyAsync(vec.data(), src, sizeof(vec[0]) * count,
                                   hipMemcpyDeviceToHost, s));
      };
      if (d->kind == BCHAR_MESH_SIMPLEX) {
        BCHAR_REQUIRE(d->vertices != nullptr && d->cells != nullptr && d->n_vertices > 0 &&
                          d->n_simplices > 0,
                      BCHAR_E_INVALID_ARG, "vertices / cells");
        down(h_vtx, d->vertices, (size_t)d->n_vertices * d->dim);
        down(h_cells, d->cells, (size_t)d->n_simplices * (d->dim + 1));
        dh.vertices = h_vtx.data();
        dh.cells = h_cells.data();
      }
      if (custom) {
        BCHAR_REQUIRE(d->balls != nullptr && d->ball_cell != nullptr && d->n_balls > 0,
                      BCHAR_E_INVALID_ARG, "CUSTOM layout: balls / ball_cell / n_balls");
        down(h_balls, d->balls, (size_t)d->n_balls * (d->dim + 1));
        down(h_bcell, d->ball_cell, (size_t)d->n_balls);
        dh.balls = h_balls.data();
        dh.ball_cell = h_bcell.data();
      }
      BCHAR_HIP(hipStreamSynchronize(s));
      d = &dh;
    }
    BCHAR_REQUIRE(d->hash_scale == 0.0 || (d->hash_scale >= 0.25 && d->hash_scale <= 4.0),
                  BCHAR_E_INVALID_ARG, "hash_scale must be 0 or within [0.25, 4]");
    auto* m = new bchar_mesh_s();
    try {
      m->hash_scale = d->hash_scale == 0.0 ? 1.0 : d->hash_scale;
      m->dim = d->dim;
      m->layout = d->layout;
      m->kind = d->kind;
      const int dim = d->dim;
      int64_t nc = 1;
      bchar::UniformBalls ub{};
      std::vector<double> kvol;   // simplex: |K| per cell
      SimplexHost sh;
      std::vector<double> pballs;     // PACKED: the balls, CUSTOM format
      std::vector<int32_t> pcell;
      if (d->kind == BCHAR_MESH_CARTESIAN) {
        double hmin = 1e300;
        ub.cell_vol = 1.0;
        for (int a = 0; a < 3; ++a) {
          if (a < dim) {
            BCHAR_REQUIRE(d->n[a] >= 1, BCHAR_E_INVALID_ARG, "n must be >= 1");
            BCHAR_REQUIRE(d->h[a] > 0 && std::isfinite(d->h[a]) && std::isfinite(d->origin[a]),
                          BCHAR_E_INVALID_ARG, "h must be finite and > 0");
            m->n[a] = d->n[a];
            m->h[a] = d->h[a];
            m->origin[a] = d->origin[a];
            nc *= d->n[a];
            hmin = std::min(hmin, d->h[a]);
            ub.cell_vol *= d->h[a];
          } else {
            m->n[a] = 1;
            m->h[a] = 1;
            m->origin[a] = 0;
          }
          m->box_lo[a] = m->origin[a];
          m->box_hi[a] = m->origin[a] + (double)m->n[a] * m->h[a];
        }
        m->n_cells = nc;
        BCHAR_REQUIRE(!packed, BCHAR_E_INVALID_ARG,
                      "PACKED is a simplex layout (SUBCELL packs Cartesian cells)");
        BCHAR_REQUIRE(d->n_ghost >= 0, BCHAR_E_INVALID_ARG, "n_ghost must be >= 0");
        for (int a = 0; a < dim; ++a)
          BCHAR_REQUIRE(d->n[a] > 2 * d->n_ghost, BCHAR_E_INVALID_ARG,
                        "n_ghost layers leave no interior cell");
        m->n_ghost = d->n_ghost;
        if (custom) {
          m->nbpc = 0;
          ub.r = 0;
        } else if (d->layout == BCHAR_LAYOUT_SUBCELL) {
          m->nbpc = 1 << dim;
          ub.r = hmin / 4.0;
        } else if (d->layout == BCHAR_LAYOUT_INSCRIBED) {
          m->nbpc = 1;
          ub.r = hmin / 2.0;
        } else {
          m->nbpc = 1;
          ub.r = dim == 2 ? std::sqrt(ub.cell_vol / kPi)
                          : cbrt_nearest(3.0 * ub.cell_vol / (4.0 * kPi));
        }
        ub.ball_vol = dim == 2 ? kPi * ub.r * ub.r : 4.0 / 3.0 * kPi * ub.r * ub.r * ub.r;
        // rho_K sum_s |B_{K,s}|_phi = |K|_phi with |B|_phi = phi_K |B|
        if (!custom) ub.rho = ub.cell_vol / (m->nbpc * ub.ball_vol);
        kvol.assign(nc, ub.cell_vol);
      } else {
        BCHAR_REQUIRE(d->layout == BCHAR_LAYOUT_EQUAL_MEASURE || custom || packed,
                      BCHAR_E_INVALID_ARG,
                      "simplicial meshes take the EQUAL_MEASURE, PACKED or CUSTOM layout");
        BCHAR_REQUIRE(d->n_ghost == 0, BCHAR_E_INVALID_ARG,
                      "ghost cells are built for Cartesian meshes");
        BCHAR_REQUIRE(d->vertices != nullptr && d->cells != nullptr, BCHAR_E_INVALID_ARG,
                      "vertices or cells is NULL");
        BCHAR_REQUIRE(d->n_vertices >= dim + 1 && d->n_simplices >= 1 &&
                          d->n_simplices < ((int64_t)1 << 31) - 1,
                      BCHAR_E_INVALID_ARG, "n_vertices / n_simplices");
        nc = d->n_simplices;
        m->n_cells = nc;
        m->nbpc = custom || packed ? 0 : 1;
        simplex_geometry(d, sh);
        for (int a = 0; a < 3; ++a) {
          m->box_lo[a] = sh.lo[a];
          m->box_hi[a] = sh.hi[a];
        }
        kvol = sh.vol;
        if (packed) packed_simplex_balls(sh, pballs, pcell);
      }
      m->n_balls = custom ? d->n_balls : (packed ? (int64_t)pcell.size() : nc * m->nbpc);
      BCHAR_REQUIRE(m->n_balls < ((int64_t)1 << 31) - 1, BCHAR_E_UNSUPPORTED,
                    "more than 2^31 balls");
      // phi: validate on the host
      std::vector<double> hphi(nc);
      if (d->phi_mem == BCHAR_MEM_HOST) {
        std::memcpy(hphi.data(), d->phi, sizeof(double) * nc);
      } else {
        BCHAR_HIP(hipMemcpyAsync(hphi.data(), d->phi, sizeof(double) * nc,
                                 hipMemcpyDeviceToHost, s));
        BCHAR_HIP(hipStreamSynchronize(s));
      }
      double pmax = 0;
      bool same = true;
      for (int64_t i = 0; i < nc; ++i) {
        BCHAR_REQUIRE(std::isfinite(hphi[i]) && hphi[i] > 0, BCHAR_E_INVALID_ARG,
                      "phi must be finite and > 0 on every cell");
        pmax = std::max(pmax, hphi[i]);
        same = same && hphi[i] == hphi[0];
      }
      m->phi_const = same;
      m->phi0 = hphi[0];
      m->phi.reserve(sizeof(double) * nc);
      BCHAR_HIP(hipMemcpyAsync(m->phi.p, hphi.data(), sizeof(double) * nc,
                               hipMemcpyHostToDevice, s));
      std::vector<uint8_t> hghost;
      if (m->n_ghost > 0) {
        // cells within n_ghost of the grid's boundary (ids x-fastest)
        hghost.assign(nc, 0);
        const int64_t g = m->n_ghost;
        for (int64_t K = 0; K < nc; ++K) {
          const int64_t idx[3] = {K % m->n[0], (K / m->n[0]) % m->n[1],
                                  K / (m->n[0] * m->n[1])};
          bool gh = false;
          for (int a = 0; a < dim; ++a) gh = gh || idx[a] < g || idx[a] >= m->n[a] - g;
          hghost[K] = gh ? 1 : 0;
        }
        m->ghost.reserve(nc);
        BCHAR_HIP(hipMemcpyAsync(m->ghost.p, hghost.data(), nc, hipMemcpyHostToDevice, s));
        BCHAR_HIP(hipStreamSynchronize(s));
      }
      if (d->kind == BCHAR_MESH_CARTESIAN && !custom) {
        m->bmax = pmax * ub.cell_vol;
        bchar::mesh_build_cartesian(m, ub, s);
      } else {
        // |K|_phi on the host (the same product phi_K |K| as on the device)
        std::vector<double> b(nc);
        m->bmax = 0;
        for (int64_t K = 0; K < nc; ++K) {
          b[K] = hphi[K] * kvol[K];
          m->bmax = std::max(m->bmax, b[K]);
        }
        if (d->kind == BCHAR_MESH_SIMPLEX) {
          simplex_upload(m, sh, b, !custom && !packed, s);
        } else {
          m->b.reserve(sizeof(double) * nc);
          BCHAR_HIP(hipMemcpyAsync(m->b.p, b.data(), sizeof(double) * nc, hipMemcpyHostToDevice,
                                   s));
        }
        if (custom) custom_layout(m, d->n_balls, d->balls, d->ball_cell, kvol, s);
        if (packed)
          custom_layout(m, (int64_t)pcell.size(), pballs.data(), pcell.data(), kvol, s);
        bchar::mesh_build_hash(m, s);
      }
    } catch (...) {
      bchar_mesh_destroy(m);
      throw;
    }
    *out = m;
    return BCHAR_OK;
  });
}

bchar_status bchar_mesh_destroy(bchar_mesh m) {
  if (!m) return BCHAR_OK;
  (void)hipDeviceSynchronize();
  m->phi.release();
  m->ghost.release();
  m->b.release();
  m->cen.release();
  m->cen32.release();
  m->bucket_start.release();
  m->bk_cen.release();
  m->bk_cen32.release();
  m->bk_ball.release();
  m->bk_rad.release();
  m->bk_cell.release();
  m->bk_w.release();
  m->ball_ptr.release();
  m->ball_cell.release();
  m->tile_cell.release();
  m->cell_cen.release();
  m->rho.release();
  m->rad.release();
  m->bvol.release();
  m->vtx.release();
  m->cells.release();
  m->pl_start.release();
  m->pl_list.release();
  m->ws.release();
  m->scratch_small.release();
  delete m;
  return BCHAR_OK;
}

bchar_status bchar_mesh_info(bchar_mesh m, int64_t* n_cells, int64_t* n_balls,
                             int* balls_per_cell) {
  if (!m) {
    bchar::set_error("mesh is NULL");
    return BCHAR_E_INVALID_ARG;
  }
  if (n_cells) *n_cells = m->n_cells;
  if (n_balls) *n_balls = m->n_balls;
  if (balls_per_cell) *balls_per_cell = m->nbpc;
  return BCHAR_OK;
}

static void transfer_free(bchar_transfer t) {
  t->row_ptr.release();
  t->col.release();
  t->V.release();
  t->AN.release();
  t->A.release();
  t->x.release();
  t->mu.release();
  t->nu.release();
  t->zdual.release();
  t->tracked.release();
  t->r_hat.release();
  t->pair_a.release();
  t->pair_b.release();
  t->stage_col.release();
  t->stage_val.release();
  t->ws.release();
  t->cscratch.release();
}

bchar_status bchar_build_transfer(bchar_mesh m, const bchar_velocity* u, double dt,
                                  const bchar_opts* opts, void* stream, bchar_transfer* out,
                                  bchar_stats* stats) {
  if (out) *out = nullptr;
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(m != nullptr && out != nullptr, BCHAR_E_INVALID_ARG, "NULL argument");
    bchar_opts o;
    opts_or_default(opts, o);
    auto* t = new bchar_transfer_s();
    t->mesh = m;
    bchar_status rc;
    try {
      rc = do_build(m, t, u, dt, o, as_stream(stream), stats);
    } catch (...) {
      transfer_free(t);
      delete t;
      throw;
    }
    if (rc != BCHAR_OK) {
      transfer_free(t);
      delete t;
      return rc;
    }
    *out = t;
    return BCHAR_OK;
  });
}

bchar_status bchar_rebuild_transfer(bchar_transfer t, const bchar_velocity* u, double dt,
                                    const bchar_opts* opts, void* stream, bchar_stats* stats) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(t != nullptr, BCHAR_E_INVALID_ARG, "transfer is NULL");
    bchar_opts o;
    opts_or_default(opts, o);
    return do_build(t->mesh, t, u, dt, o, as_stream(stream), stats);
  });
}

bchar_status bchar_build_transfer_tracked(bchar_mesh m, const double* tracked,
                                          const double* r_hat, const bchar_opts* opts,
                                          void* stream, bchar_transfer* out,
                                          bchar_stats* stats) {
  if (out) *out = nullptr;
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(m != nullptr && out != nullptr && tracked != nullptr && r_hat != nullptr,
                  BCHAR_E_INVALID_ARG, "NULL argument");
    bchar_opts o;
    opts_or_default(opts, o);
    validate_opts(o);
    BCHAR_REQUIRE(o.divergence == BCHAR_DIV_FREE, BCHAR_E_UNSUPPORTED,
                  "a non-solenoidal build tracks its own balls (their growth is not given)");
    hipStream_t s = as_stream(stream);
    auto* t = new bchar_transfer_s();
    t->mesh = m;
    bchar_status rc;
    try {
      t->ws.reset();
      t->tracked.reserve(sizeof(double) * m->dim * m->n_balls);
      t->r_hat.reserve(sizeof(double) * m->n_balls);
      BCHAR_HIP(hipMemcpyAsync(t->tracked.p, tracked, sizeof(double) * m->dim * m->n_balls,
                               hipMemcpyDeviceToDevice, s));
      BCHAR_HIP(hipMemcpyAsync(t->r_hat.p, r_hat, sizeof(double) * m->n_balls,
                               hipMemcpyDeviceToDevice, s));
      rc = build_from_tracked(m, t, o, BCHAR_FP64, s, stats);
    } catch (...) {
      transfer_free(t);
      delete t;
      throw;
    }
    if (rc != BCHAR_OK) {
      transfer_free(t);
      delete t;
      return rc;
    }
    *out = t;
    return BCHAR_OK;
  });
}

bchar_status bchar_build_transfer_batch(bchar_build_job* jobs, int n_jobs,
                                        const bchar_opts* opts, void* const* streams,
                                        int n_streams) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(n_jobs >= 0 && (n_jobs == 0 || jobs != nullptr) && n_streams >= 1 &&
                      streams != nullptr,
                  BCHAR_E_INVALID_ARG, "NULL argument or n_streams < 1");
    std::set<bchar_transfer> seen;
    for (int i = 0; i < n_jobs; ++i) {
      BCHAR_REQUIRE(jobs[i].transfer != nullptr || jobs[i].mesh != nullptr,
                    BCHAR_E_INVALID_ARG, "job without transfer and mesh");
      if (jobs[i].transfer)
        BCHAR_REQUIRE(seen.insert(jobs[i].transfer).second, BCHAR_E_INVALID_ARG,
                      "a transfer appears in two jobs");
    }
    // warm starts from other transfers, taken before any job runs (the
    // source may itself be rebuilt by a job of this batch)
    {
      hipStream_t s0 = as_stream(streams[0]);
      bool copied = false;
      for (int i = 0; i < n_jobs; ++i) {
        bchar_transfer_s* dst = jobs[i].transfer;
        const bchar_transfer_s* src = jobs[i].warm_from;
        if (!src || !dst || src == dst) continue;
        BCHAR_REQUIRE(src->mesh == dst->mesh, BCHAR_E_INVALID_ARG,
                      "warm_from is a transfer of another mesh");
        // the leading parts of the multipliers (the compensation restarts
        // with a warm start); the transfer keeps both parts, 4 n values
        const size_t bytes = sizeof(double) * 2 * dst->mesh->n_cells;
        if (src->warm_level < 0 || src->zdual.bytes < bytes) continue;
        if (dst->zdual.bytes < 2 * bytes) dst->zdual.reserve(2 * bytes);
        BCHAR_HIP(hipMemcpyAsync(dst->zdual.p, src->zdual.p, bytes, hipMemcpyDeviceToDevice, s0));
        dst->warm_level = src->warm_level;
        dst->warm_newton_skip = src->warm_newton_skip;
        copied = true;
      }
      if (copied) BCHAR_HIP(hipStreamSynchronize(s0));
    }
    int dev = 0;
    BCHAR_HIP(hipGetDevice(&dev));
    std::vector<std::string> msg(n_jobs);
    const int workers = std::min(n_streams, std::max(n_jobs, 1));
    std::vector<hipError_t> sync_err(workers, hipSuccess);
    // jobs are taken in index order from a shared counter, each by the
    // first worker that is free
    std::atomic<int> next{0};
    auto run = [&](int w) {
      sync_err[w] = hipSetDevice(dev);
      for (int i = next++; i < n_jobs; i = next++) {
        bchar_build_job& J = jobs[i];
        if (sync_err[w] != hipSuccess) {
          J.status = BCHAR_E_DEVICE;
          msg[i] = "hipSetDevice failed in a worker";
          continue;
        }
        J.status = J.transfer ? bchar_rebuild_transfer(J.transfer, J.u, J.dt, opts, streams[w],
                                                       &J.stats)
                              : bchar_build_transfer(J.mesh, J.u, J.dt, opts, streams[w],
                                                     &J.transfer, &J.stats);
        if (J.status != BCHAR_OK) msg[i] = bchar_last_error();
      }
      if (sync_err[w] == hipSuccess) sync_err[w] = hipStreamSynchronize(as_stream(streams[w]));
    };
    std::vector<std::thread> pool;
    for (int w = 1; w < workers; ++w) pool.emplace_back(run, w);
    run(0);
    for (auto& th : pool) th.join();
    for (int w = 0; w < workers; ++w) BCHAR_HIP(sync_err[w]);
    for (int i = 0; i < n_jobs; ++i)
      if (jobs[i].status != BCHAR_OK) {
        bchar::set_error("job " + std::to_string(i) + ": " + msg[i]);
        return jobs[i].status;
      }
    return BCHAR_OK;
  });
}

bchar_status bchar_tune_options(const bchar_build_job* jobs, int n_jobs,
                                const bchar_opts* candidates, int n_candidates, int rounds,
                                void* const* streams, int n_streams, int* best,
                                double* seconds) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(jobs != nullptr && n_jobs >= 1 && candidates != nullptr && n_candidates >= 1 &&
                      rounds >= 1 && streams != nullptr && n_streams >= 1 && best != nullptr,
                  BCHAR_E_INVALID_ARG, "NULL argument or a count < 1");
    for (int i = 0; i < n_jobs; ++i)
      BCHAR_REQUIRE(jobs[i].transfer == nullptr && jobs[i].warm_from == nullptr &&
                        jobs[i].mesh != nullptr && jobs[i].u != nullptr,
                    BCHAR_E_INVALID_ARG, "a tuning job names a mesh and a velocity, no transfer");
    for (int c = 0; c < n_candidates; ++c) validate_opts(candidates[c]);
    std::vector<bchar_build_job> J(n_jobs);
    // one batch: fresh transfers, built and destroyed; its status
    auto batch = [&](const bchar_opts& o) -> bchar_status {
      for (int i = 0; i < n_jobs; ++i) {
        J[i] = jobs[i];
        J[i].transfer = nullptr;
      }
      const bchar_status st = bchar_build_transfer_batch(J.data(), n_jobs, &o, streams, n_streams);
      for (auto& j : J)
        if (j.transfer) bchar_transfer_destroy(j.transfer);
      return st;
    };
    // untimed: device buffers, code and caches warmed once
    (void)batch(candidates[0]);
    std::vector<double> total(n_candidates, 0.0);
    std::vector<bchar_status> failed(n_candidates, BCHAR_OK);
    std::string first_msg;
    for (int r = 0; r < rounds; ++r)
      for (int k = 0; k < n_candidates; ++k) {
        const int c = (r % 2 == 0) ? k : n_candidates - 1 - k;
        if (failed[c] != BCHAR_OK) continue;
        const double t0 = bchar::wall_seconds();
        const bchar_status st = batch(candidates[c]);
        const double t = bchar::wall_seconds() - t0;
        if (st != BCHAR_OK) {
          failed[c] = st;
          if (first_msg.empty()) first_msg = bchar_last_error();
          continue;
        }
        total[c] += t;
      }
    int b = -1;
    for (int c = 0; c < n_candidates; ++c) {
      if (seconds) seconds[c] = failed[c] == BCHAR_OK ? total[c] : HUGE_VAL;
      if (failed[c] == BCHAR_OK && (b < 0 || total[c] < total[b])) b = c;
    }
    if (b < 0) {
      bchar::set_error("every candidate failed: " + first_msg);
      return failed[0];
    }
    *best = b;
    return BCHAR_OK;
  });
}

bchar_status bchar_transfer_destroy(bchar_transfer t) {
  if (!t) return BCHAR_OK;
  (void)hipDeviceSynchronize();
  transfer_free(t);
  delete t;
  return BCHAR_OK;
}

bchar_status bchar_step(bchar_transfer t, const double* cin, double* cout, void* stream) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(t != nullptr && cin != nullptr && cout != nullptr, BCHAR_E_INVALID_ARG,
                  "NULL argument");
    BCHAR_REQUIRE(t->stage == BCHAR_STAGE_ALL, BCHAR_E_INVALID_ARG,
                  "transfer was not built to the final stage");
    const int64_t n = t->mesh->n_cells;
    const double* ce = cin + n;
    BCHAR_REQUIRE(cout + n <= cin || ce <= cout, BCHAR_E_INVALID_ARG,
                  "c_in and c_out overlap");
    if (t->substeps > 1) t->cscratch.reserve(sizeof(double) * n);
    apply_substeps(t, cin, cout, t->cscratch.as<double>(), as_stream(stream));
    return BCHAR_OK;
  });
}

bchar_status bchar_mass(bchar_mesh m, const double* c, void* stream, double* host_out) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(m != nullptr && c != nullptr && host_out != nullptr, BCHAR_E_INVALID_ARG,
                  "NULL argument");
    *host_out = bchar::porous_mass(m, c, m->ws, as_stream(stream));
    return BCHAR_OK;
  });
}

bchar_status bchar_mass_into(bchar_mesh m, const double* c, double* d_out, void* stream) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(m != nullptr && c != nullptr && d_out != nullptr, BCHAR_E_INVALID_ARG,
                  "NULL argument");
    BCHAR_REQUIRE(m->n_cells <= kMassIntoMaxCells, BCHAR_E_INVALID_ARG,
                  "bchar_mass_into takes at most 2^31 - 1 cells");
    bchar::porous_mass_into(m, c, d_out, as_stream(stream));
    return BCHAR_OK;
  });
}

bchar_status bchar_transfer_info(bchar_transfer t, int64_t* n_rows, int64_t* nnz,
                                 int64_t* n_pairs, int* stage) {
  if (!t) {
    bchar::set_error("transfer is NULL");
    return BCHAR_E_INVALID_ARG;
  }
  if (n_rows) *n_rows = t->mesh->n_cells;
  if (nnz) *nnz = t->nnz;
  if (n_pairs) *n_pairs = t->n_pairs;
  if (stage) *stage = t->stage;
  return BCHAR_OK;
}

bchar_status bchar_transfer_export_csr(bchar_transfer t, int stage, int64_t* row_ptr,
                                       int32_t* col, double* val) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(t != nullptr, BCHAR_E_INVALID_ARG, "transfer is NULL");
    BCHAR_REQUIRE(stage >= BCHAR_STAGE_V && stage <= BCHAR_STAGE_ALL && stage <= t->stage,
                  BCHAR_E_INVALID_ARG, "stage not built");
    const int64_t n = t->mesh->n_cells;
    BCHAR_HIP(hipDeviceSynchronize());
    if (row_ptr) {
      std::vector<int32_t> rp(n + 1);
      BCHAR_HIP(hipMemcpy(rp.data(), t->row_ptr.p, sizeof(int32_t) * (n + 1),
                          hipMemcpyDeviceToHost));
      for (int64_t i = 0; i <= n; ++i) row_ptr[i] = rp[i];
    }
    if (col)
      BCHAR_HIP(hipMemcpy(col, t->col.p, sizeof(int32_t) * t->nnz, hipMemcpyDeviceToHost));
    if (val) {
      const bchar::DBuf& src = stage == BCHAR_STAGE_V ? t->V
                               : stage == BCHAR_STAGE_SCALING ? t->AN
                                                               : t->A;
      BCHAR_HIP(hipMemcpy(val, src.p, sizeof(double) * t->nnz, hipMemcpyDeviceToHost));
    }
    return BCHAR_OK;
  });
}

bchar_status bchar_transfer_export_pairs(bchar_transfer t, int32_t* tracked, int32_t* residing) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(t != nullptr && tracked != nullptr && residing != nullptr,
                  BCHAR_E_INVALID_ARG, "NULL argument");
    BCHAR_REQUIRE(t->pair_a.p != nullptr && t->stage >= BCHAR_STAGE_V, BCHAR_E_INVALID_ARG,
                  "pairs were not kept (opts.keep_pairs)");
    const int64_t np = t->n_pairs;
    BCHAR_HIP(hipDeviceSynchronize());
    std::vector<int32_t> a(np), b(np);
    BCHAR_HIP(hipMemcpy(a.data(), t->pair_a.p, sizeof(int32_t) * np, hipMemcpyDeviceToHost));
    BCHAR_HIP(hipMemcpy(b.data(), t->pair_b.p, sizeof(int32_t) * np, hipMemcpyDeviceToHost));
    std::vector<int64_t> idx(np);
    for (int64_t i = 0; i < np; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
      return a[x] != a[y] ? a[x] < a[y] : b[x] < b[y];
    });
    for (int64_t i = 0; i < np; ++i) {
      tracked[i] = a[idx[i]];
      residing[i] = b[idx[i]];
    }
    return BCHAR_OK;
  });
}

bchar_status bchar_transfer_export_tracked(bchar_transfer t, double* tracked, double* r_hat) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(t != nullptr, BCHAR_E_INVALID_ARG, "transfer is NULL");
    const bchar_mesh_s* m = t->mesh;
    BCHAR_HIP(hipDeviceSynchronize());
    if (tracked)
      BCHAR_HIP(hipMemcpy(tracked, t->tracked.p, sizeof(double) * m->dim * m->n_balls,
                          hipMemcpyDeviceToHost));
    if (r_hat)
      BCHAR_HIP(hipMemcpy(r_hat, t->r_hat.p, sizeof(double) * m->n_balls,
                          hipMemcpyDeviceToHost));
    return BCHAR_OK;
  });
}

bchar_status bchar_transfer_export_targets(bchar_transfer t, double* lam, double* b_row) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(t != nullptr, BCHAR_E_INVALID_ARG, "transfer is NULL");
    const bchar_mesh_s* m = t->mesh;
    BCHAR_HIP(hipDeviceSynchronize());
    if (lam) {
      if (t->general)
        BCHAR_HIP(hipMemcpy(lam, t->lam.p, sizeof(double) * m->n_balls, hipMemcpyDeviceToHost));
      else
        for (int64_t i = 0; i < m->n_balls; ++i) lam[i] = 0.0;
    }
    if (b_row)
      BCHAR_HIP(hipMemcpy(b_row, t->general ? t->b_row.p : m->b.p, sizeof(double) * m->n_cells,
                          hipMemcpyDeviceToHost));
    return BCHAR_OK;
  });
}

bchar_status bchar_transfer_export_qp(bchar_transfer t, double* x, double* mu, double* nu) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(t != nullptr && t->stage == BCHAR_STAGE_ALL, BCHAR_E_INVALID_ARG,
                  "transfer not built to the final stage");
    const int64_t n = t->mesh->n_cells;
    BCHAR_HIP(hipDeviceSynchronize());
    if (x) BCHAR_HIP(hipMemcpy(x, t->x.p, sizeof(double) * t->nnz, hipMemcpyDeviceToHost));
    if (mu) BCHAR_HIP(hipMemcpy(mu, t->mu.p, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (nu) BCHAR_HIP(hipMemcpy(nu, t->nu.p, sizeof(double) * n, hipMemcpyDeviceToHost));
    return BCHAR_OK;
  });
}

bchar_status bchar_transfer_export_qp_dual(bchar_transfer t, double* sv, double* gv,
                                           double* s_lo, double* g_lo) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(t != nullptr && t->stage == BCHAR_STAGE_ALL, BCHAR_E_INVALID_ARG,
                  "transfer not built to the final stage");
    const int64_t n = t->mesh->n_cells;
    BCHAR_HIP(hipDeviceSynchronize());
    const double* z = t->zdual.as<double>();
    double* out[4] = {sv, gv, s_lo, g_lo};
    for (int i = 0; i < 4; ++i)
      if (out[i])
        BCHAR_HIP(hipMemcpy(out[i], z + i * n, sizeof(double) * n, hipMemcpyDeviceToHost));
    return BCHAR_OK;
  });
}

bchar_status bchar_mesh_export_balls(bchar_mesh m, double* centres, double* radii,
                                     int32_t* cell) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(m != nullptr, BCHAR_E_INVALID_ARG, "mesh is NULL");
    BCHAR_HIP(hipDeviceSynchronize());
    if (centres)
      BCHAR_HIP(hipMemcpy(centres, m->cen.p, sizeof(double) * m->dim * m->n_balls,
                          hipMemcpyDeviceToHost));
    if (radii)
      BCHAR_HIP(hipMemcpy(radii, m->rad.p, sizeof(double) * m->n_balls, hipMemcpyDeviceToHost));
    if (cell && m->nbpc > 0)
      for (int64_t b = 0; b < m->n_balls; ++b) cell[b] = (int32_t)(b / m->nbpc);
    else if (cell)
      BCHAR_HIP(hipMemcpy(cell, m->ball_cell.p, sizeof(int32_t) * m->n_balls,
                          hipMemcpyDeviceToHost));
    return BCHAR_OK;
  });
}

bchar_status bchar_server_create(int n_workers, void* const* streams, int64_t mem_budget,
                                 const bchar_opts* opts, bchar_server* out) {
  if (out) *out = nullptr;
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(out != nullptr && streams != nullptr && n_workers >= 1 && mem_budget >= 0,
                  BCHAR_E_INVALID_ARG, "NULL argument, n_workers < 1 or mem_budget < 0");
    auto* srv = new bchar_server_s();
    opts_or_default(opts, srv->opts);
    validate_opts(srv->opts);
    BCHAR_HIP(hipGetDevice(&srv->dev));
    srv->budget = mem_budget;
    srv->retained.assign(n_workers, 0);
    for (int w = 0; w < n_workers; ++w) {
      srv->streams.push_back(as_stream(streams[w]));
      srv->transfers.push_back(new bchar_transfer_s());
    }
    for (int w = 0; w < n_workers; ++w) srv->workers.emplace_back(&bchar_server_s::work, srv, w);
    *out = srv;
    return BCHAR_OK;
  });
}

bchar_status bchar_server_submit(bchar_server srv, const bchar_request* req, int64_t* ticket) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(srv != nullptr && req != nullptr && ticket != nullptr, BCHAR_E_INVALID_ARG,
                  "NULL argument");
    BCHAR_REQUIRE(req->mesh != nullptr && req->u != nullptr && req->c_in != nullptr &&
                      req->c_out != nullptr && req->steps >= 1 &&
                      (req->steps == 1 || req->c_tmp != nullptr),
                  BCHAR_E_INVALID_ARG, "request: NULL pointer, steps < 1 or no c_tmp");
    std::lock_guard<std::mutex> lk(srv->mu);
    BCHAR_REQUIRE(!srv->stopping, BCHAR_E_INVALID_ARG, "server is being destroyed");
    const int64_t id = srv->next_ticket++;
    bchar_server_s::Item& it = srv->items[id];
    it.req = *req;
    it.bytes = req->bytes > 0 ? req->bytes : 900 * req->mesh->n_balls;
    it.res.t_submit = bchar::wall_seconds();
    srv->queue.push_back(id);
    *ticket = id;
    srv->cv.notify_all();
    return BCHAR_OK;
  });
}

bchar_status bchar_server_wait(bchar_server srv, int64_t ticket, bchar_request_result* res) {
  return guarded([&]() -> bchar_status {
    BCHAR_REQUIRE(srv != nullptr && res != nullptr, BCHAR_E_INVALID_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto f = srv->items.find(ticket);
    BCHAR_REQUIRE(f != srv->items.end(), BCHAR_E_INVALID_ARG, "unknown ticket");
    srv->cv.wait(lk, [&] { return f->second.done; });
    *res = f->second.res;
    srv->items.erase(f);
    return BCHAR_OK;
  });
}

bchar_status bchar_server_destroy(bchar_server srv) {
  if (!srv) return BCHAR_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
  }
  srv->cv.notify_all();
  for (auto& th : srv->workers) th.join();
  for (auto* t : srv->transfers) {
    transfer_free(t);
    delete t;
  }
  delete srv;
  return BCHAR_OK;
}

}  // extern "C"
