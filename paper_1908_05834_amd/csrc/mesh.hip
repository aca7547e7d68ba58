// Mesh-static data: balls of every cell (Sec. 3) and the spatial hash.
//
// The balls of a Cartesian cell follow the layout chosen at creation
// (see bchar.h); those of a simplicial mesh come from the host (one
// centroid ball per cell).  Residing balls are bucketed on a uniform grid
// of side hs = 2 r_max over the domain box (times the mesh's hash_scale),
// so that every ball overlapping a tracked ball of radius r_hat <= r_max
// lies in the 3^d buckets around the tracked centre; larger tracked radii
// or smaller buckets widen the searched block (build.hip).  Bucket contents (centres, binary64 and binary32, and
// radii) are stored contiguously in bucket order (SoA) so that a query
// streams them.
#include "device_util.hpp"
#include "internal.hpp"

namespace bchar {

// Ball b of cell K = b / nbpc, sub-ball s = b % nbpc: centre per layout.
__global__ void k_ball_centres(int dim, int nbpc, int64_t n0, int64_t n1, int64_t n_balls,
                               double o0, double o1, double o2, double h0, double h1,
                               double h2, double* __restrict__ cen, float* __restrict__ cen32) {
#pragma clang fp contract(off)
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_balls) return;
  const int64_t K = b / nbpc;
  const int s = (int)(b % nbpc);
  const int64_t i = K % n0;
  const int64_t j = (K / n0) % n1;
  const int64_t k = K / (n0 * n1);
  double f0, f1, f2;
  if (nbpc == 1) {
    f0 = f1 = f2 = 0.5;
  } else {
    // sub-cell centres at 1/4 and 3/4 of the cell along each axis
    f0 = (s & 1) ? 0.75 : 0.25;
    f1 = (s & 2) ? 0.75 : 0.25;
    f2 = (s & 4) ? 0.75 : 0.25;
  }
  const double x = o0 + ((double)i + f0) * h0;
  const double y = o1 + ((double)j + f1) * h1;
  cen[b] = x;
  cen[n_balls + b] = y;
  cen32[b] = (float)x;
  cen32[n_balls + b] = (float)y;
  if (dim == 3) {
    const double z = o2 + ((double)k + f2) * h2;
    cen[2 * n_balls + b] = z;
    cen32[2 * n_balls + b] = (float)z;
  }
}

__global__ void k_bucket_of(int dim, int64_t n_balls, const double* __restrict__ cen,
                            double o0, double o1, double o2, double inv_hs, int64_t nb0,
                            int64_t nb1, int64_t nb2, int32_t* __restrict__ key) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_balls) return;
  int64_t i0 = (int64_t)floor((cen[b] - o0) * inv_hs);
  int64_t i1 = (int64_t)floor((cen[n_balls + b] - o1) * inv_hs);
  i0 = i0 < 0 ? 0 : (i0 >= nb0 ? nb0 - 1 : i0);
  i1 = i1 < 0 ? 0 : (i1 >= nb1 ? nb1 - 1 : i1);
  int64_t i2 = 0;
  if (dim == 3) {
    i2 = (int64_t)floor((cen[2 * n_balls + b] - o2) * inv_hs);
    i2 = i2 < 0 ? 0 : (i2 >= nb2 ? nb2 - 1 : i2);
  }
  key[b] = (int32_t)(i0 + nb0 * (i1 + nb1 * i2));
}

__global__ void k_gather_bucketed(int dim, int64_t n_balls, const int32_t* __restrict__ perm,
                                  const double* __restrict__ cen,
                                  const float* __restrict__ cen32,
                                  const double* __restrict__ rad, double* __restrict__ bk,
                                  float* __restrict__ bk32, double* __restrict__ bkr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_balls) return;
  const int64_t b = perm[p];
  for (int a = 0; a < dim; ++a) {
    bk[a * n_balls + p] = cen[a * n_balls + b];
    bk32[a * n_balls + p] = cen32[a * n_balls + b];
  }
  bkr[p] = rad[b];
}

// Cell and weight rho_M phi_M of every bucket slot (the residing ball's
// cell: ball / nbpc, or the per-ball cell of a varying layout).
__global__ void k_slot_cells(int64_t n_balls, int nbpc, const int32_t* __restrict__ ball_cell,
                             const int32_t* __restrict__ bk_ball, const double* __restrict__ rho,
                             const double* __restrict__ phi, int32_t* __restrict__ bk_cell,
                             double* __restrict__ bk_w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_balls) return;
  const int32_t b = bk_ball[e];
  const int32_t M = nbpc > 0 ? b / nbpc : ball_cell[b];
  bk_cell[e] = M;
  bk_w[e] = rho[M] * phi[M];
}

__global__ void k_porous_volume(const double* __restrict__ phi, double vol, int64_t n,
                                double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = phi[i] * vol;
}

void mesh_build_cartesian(bchar_mesh_s* m, const UniformBalls& u, hipStream_t s) {
  const int64_t nb = m->n_balls;
  m->cen.reserve(sizeof(double) * m->dim * nb);
  m->cen32.reserve(sizeof(float) * m->dim * nb);
  {
    ::bchar::ProfScope ps_("k_ball_centres", s);
    k_ball_centres<<<blocks_for(nb, 256), 256, 0, s>>>(
        m->dim, m->nbpc, m->n[0], m->n[1], nb, m->origin[0], m->origin[1], m->origin[2], m->h[0],
        m->h[1], m->h[2], m->cen.as<double>(), m->cen32.as<float>());
  }
  BCHAR_HIP(hipGetLastError());
  m->b.reserve(sizeof(double) * m->n_cells);
  {
    ::bchar::ProfScope ps_("k_porous_volume", s);
    k_porous_volume<<<blocks_for(m->n_cells, 256), 256, 0, s>>>(
        m->phi.as<double>(), u.cell_vol, m->n_cells, m->b.as<double>());
  }
  BCHAR_HIP(hipGetLastError());
  m->rad.reserve(sizeof(double) * nb);
  m->bvol.reserve(sizeof(double) * nb);
  m->rho.reserve(sizeof(double) * m->n_cells);
  fill_f64(m->rad.as<double>(), u.r, nb, s);
  fill_f64(m->bvol.as<double>(), u.ball_vol, nb, s);
  fill_f64(m->rho.as<double>(), u.rho, m->n_cells, s);
  m->rmax = u.r;
  m->r_uniform = true;
  m->r0 = u.r;
  mesh_build_hash(m, s);
}

void mesh_build_hash(bchar_mesh_s* m, hipStream_t s) {
  const int64_t nb = m->n_balls;
  // uniform bucket grid of side 2 r_max (times hash_scale) over the domain box
  m->hs = 2.0 * m->rmax * m->hash_scale;
  m->n_buckets = 1;
  for (int a = 0; a < 3; ++a) {
    if (a < m->dim) {
      double L = m->box_hi[a] - m->box_lo[a];
      int64_t c = (int64_t)ceil(L / m->hs);
      m->nbk[a] = c < 1 ? 1 : c;
    } else {
      m->nbk[a] = 1;
    }
    m->n_buckets *= m->nbk[a];
  }
  BCHAR_REQUIRE(m->n_buckets < (int64_t)1 << 31, BCHAR_E_UNSUPPORTED,
                "too many hash buckets for 32-bit indices");
  m->ws.reset();
  int32_t* key = m->ws.get<int32_t>(nb);
  {
    ::bchar::ProfScope ps_("k_bucket_of", s);
    k_bucket_of<<<blocks_for(nb, 256), 256, 0, s>>>(
        m->dim, nb, m->cen.as<double>(), m->box_lo[0], m->box_lo[1], m->box_lo[2], 1.0 / m->hs,
        m->nbk[0], m->nbk[1], m->nbk[2], key);
  }
  BCHAR_HIP(hipGetLastError());
  m->bucket_start.reserve(sizeof(int32_t) * (m->n_buckets + 1));
  m->bk_ball.reserve(sizeof(int32_t) * nb);
  bucket_sort(key, nb, m->n_buckets, m->bucket_start.as<int32_t>(), m->bk_ball.as<int32_t>(),
              m->ws, s);
  m->bk_cen.reserve(sizeof(double) * m->dim * nb);
  m->bk_cen32.reserve(sizeof(float) * m->dim * nb);
  m->bk_rad.reserve(sizeof(double) * nb);
  {
    ::bchar::ProfScope ps_("k_gather_bucketed", s);
    k_gather_bucketed<<<blocks_for(nb, 256), 256, 0, s>>>(
        m->dim, nb, m->bk_ball.as<int32_t>(), m->cen.as<double>(), m->cen32.as<float>(),
        m->rad.as<double>(), m->bk_cen.as<double>(), m->bk_cen32.as<float>(),
        m->bk_rad.as<double>());
  }
  BCHAR_HIP(hipGetLastError());
  m->bk_cell.reserve(sizeof(int32_t) * nb);
  m->bk_w.reserve(sizeof(double) * nb);
  {
    ::bchar::ProfScope ps_("k_slot_cells", s);
    k_slot_cells<<<blocks_for(nb, 256), 256, 0, s>>>(
        nb, m->nbpc, m->ball_cell.as<int32_t>(), m->bk_ball.as<int32_t>(), m->rho.as<double>(),
        m->phi.as<double>(), m->bk_cell.as<int32_t>(), m->bk_w.as<double>());
  }
  BCHAR_HIP(hipGetLastError());
  BCHAR_HIP(hipStreamSynchronize(s));
  m->ws.reset();
}

}  // namespace bchar
