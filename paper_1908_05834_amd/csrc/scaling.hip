// Mass adjustment: N sweeps of eq. volAdj (Sec. 3.2).
//
// The sweeps only rescale rows and columns, so A^(n) = diag(R) V diag(C)
// and only the two scaling vectors change:
//     C_j <- |M_j|_phi / sum_i R_i v_ij      (columns to their porous volume)
//     R_i <- |K_i|_phi / sum_j v_ij C_j      (rows to theirs)
// Column sums run over a CSC copy of V (values laid out column-major so
// that the pass streams them), row sums over the CSR.  Sums are compensated
// (TwoSum) and each is taken by one thread in storage order: the result is
// the same on every run.
#include "device_util.hpp"
#include "internal.hpp"

namespace bchar {

__global__ void k_expand_rows(const int32_t* __restrict__ row_ptr, int64_t n,
                              int32_t* __restrict__ row_of) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) row_of[k] = (int32_t)i;
}

__global__ void k_csc_rows(const int32_t* __restrict__ perm, const int32_t* __restrict__ row_of,
                           int64_t nnz, int32_t* __restrict__ csc_row) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) csc_row[e] = row_of[perm[e]];
}

void build_csc(const int32_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz, Csc& c,
               Arena& ws, hipStream_t s) {
  c.ptr = ws.get<int32_t>(n + 1);
  c.pos = ws.get<int32_t>(nnz + 1);
  c.row = ws.get<int32_t>(nnz + 1);
  Arena::Mark mk = ws.mark();
  int32_t* row_of = ws.get<int32_t>(nnz + 1);
  {
    ::bchar::ProfScope ps_("k_expand_rows", s);
    k_expand_rows<<<blocks_for(n, 256), 256, 0, s>>>(row_ptr, n, row_of);
  }
  BCHAR_HIP(hipGetLastError());
  bucket_sort(col, nnz, n, c.ptr, c.pos, ws, s);
  {
    ::bchar::ProfScope ps_("k_csc_rows", s);
    k_csc_rows<<<blocks_for(nnz, 256), 256, 0, s>>>(c.pos, row_of, nnz, c.row);
  }
  BCHAR_HIP(hipGetLastError());
  ws.rewind(mk);
}

__global__ void k_gather_f64(const double* __restrict__ src, const int32_t* __restrict__ idx,
                             int64_t n, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = src[idx[e]];
}

// ghost (optional): cells without targets (ghost cells), left unscaled
__global__ void k_col_scale(const int32_t* __restrict__ cptr, const int32_t* __restrict__ crow,
                            const double* __restrict__ vc, const double* __restrict__ R,
                            const double* __restrict__ b, const uint8_t* __restrict__ ghost,
                            int64_t n, double* __restrict__ C, int32_t* __restrict__ void_col) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (ghost && ghost[j]) {
    C[j] = 1.0;
    return;
  }
  CSum acc;
  for (int32_t e = cptr[j]; e < cptr[j + 1]; ++e) acc.add(R[crow[e]] * vc[e]);
  const double cs = acc.value();
  if (!(cs > 0.0)) {
    atomicMin(void_col, (int32_t)j);   // void_col[0]: first void column
    atomicAdd(void_col + 1, 1);        // void_col[1]: their number
    C[j] = 0.0;
    return;
  }
  C[j] = b[j] / cs;
}

__global__ void k_row_scale(const int32_t* __restrict__ rptr, const int32_t* __restrict__ col,
                            const double* __restrict__ v, const double* __restrict__ C,
                            const double* __restrict__ b, const uint8_t* __restrict__ ghost,
                            int64_t n, double* __restrict__ R) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (ghost && ghost[i]) {
    R[i] = 1.0;
    return;
  }
  CSum acc;
  for (int32_t k = rptr[i]; k < rptr[i + 1]; ++k) acc.add(v[k] * C[col[k]]);
  const double rs = acc.value();
  R[i] = rs > 0.0 ? b[i] / rs : 0.0;
}

__global__ void k_apply_scaling(const int32_t* __restrict__ rptr, const int32_t* __restrict__ col,
                                const double* __restrict__ v, const double* __restrict__ R,
                                const double* __restrict__ C, int64_t n,
                                double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ri = R[i];
  for (int32_t k = rptr[i]; k < rptr[i + 1]; ++k) out[k] = ri * v[k] * C[col[k]];
}

// max_j |sum_i a_ij / b_j - 1| over the final matrix (CSC order)
__global__ void k_col_err(const int32_t* __restrict__ cptr, const int32_t* __restrict__ pos,
                          const double* __restrict__ a, const double* __restrict__ b,
                          const uint8_t* __restrict__ ghost, int64_t n,
                          double* __restrict__ part) {
  __shared__ double sh[16];
  double m = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    if (ghost && ghost[j]) continue;
    CSum acc;
    for (int32_t e = cptr[j]; e < cptr[j + 1]; ++e) acc.add(a[pos[e]]);
    m = fmax(m, fabs(acc.value() / b[j] - 1.0));
  }
  m = block_max(m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

bchar_status scaling_sweeps(const bchar_mesh_s* m, const int32_t* row_ptr, const int32_t* col,
                            const Csc& csc, const double* V, const double* b_row, int64_t nnz,
                            int n_sweeps, double* AN, int64_t* void_col, int64_t* n_void_cols,
                            double* max_col_err, Arena& ws, hipStream_t s) {
  const int64_t n = m->n_cells;
  const double* b = m->b.as<double>();
  const uint8_t* ghost = m->ghost.as<uint8_t>();
  Arena::Mark mk = ws.mark();
  double* vc = ws.get<double>(nnz + 1);
  double* R = ws.get<double>(n);
  double* C = ws.get<double>(n);
  int32_t* flag = ws.get<int32_t>(2);
  {
    ::bchar::ProfScope ps_("k_gather_f64", s);
    k_gather_f64<<<blocks_for(nnz, 256), 256, 0, s>>>(V, csc.pos, nnz, vc);
  }
  BCHAR_HIP(hipGetLastError());
  fill_f64(R, 1.0, n, s);
  fill_i32(flag, INT32_MAX, 1, s);
  fill_i32(flag + 1, 0, 1, s);
  // a column of V summing to zero cannot be scaled (Sec. 3.2)
  {
    ::bchar::ProfScope ps_("k_col_scale", s);
    k_col_scale<<<blocks_for(n, 256), 256, 0, s>>>(csc.ptr, csc.row, vc, R, b, ghost, n, C,
                                                    flag);
  }
  BCHAR_HIP(hipGetLastError());
  int32_t hflag[2] = {INT32_MAX, 0};
  BCHAR_HIP(hipMemcpyAsync(hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, s));
  BCHAR_HIP(hipStreamSynchronize(s));
  *n_void_cols = hflag[1];
  if (hflag[0] != INT32_MAX) {
    *void_col = hflag[0];
    ws.rewind(mk);
    return BCHAR_E_VOID_COLUMN;
  }
  for (int it = 0; it < n_sweeps; ++it) {
    if (it > 0) {
      {
        ::bchar::ProfScope ps_("k_col_scale", s);
        k_col_scale<<<blocks_for(n, 256), 256, 0, s>>>(csc.ptr, csc.row, vc, R, b, ghost, n, C,
                                                        flag);
      }
      BCHAR_HIP(hipGetLastError());
    }
    {
      ::bchar::ProfScope ps_("k_row_scale", s);
      k_row_scale<<<blocks_for(n, 256), 256, 0, s>>>(row_ptr, col, V, C, b_row, ghost, n, R);
    }
    BCHAR_HIP(hipGetLastError());
  }
  if (n_sweeps == 0) {
    fill_f64(R, 1.0, n, s);
    fill_f64(C, 1.0, n, s);
  }
  {
    ::bchar::ProfScope ps_("k_apply_scaling", s);
    k_apply_scaling<<<blocks_for(n, 256), 256, 0, s>>>(row_ptr, col, V, R, C, n, AN);
  }
  BCHAR_HIP(hipGetLastError());
  const int nb = 256;
  double* part = ws.get<double>(nb);
  {
    ::bchar::ProfScope ps_("k_col_err", s);
    k_col_err<<<nb, 256, 0, s>>>(csc.ptr, csc.pos, AN, b, ghost, n, part);
  }
  BCHAR_HIP(hipGetLastError());
  double h[nb];
  BCHAR_HIP(hipMemcpyAsync(h, part, sizeof(h), hipMemcpyDeviceToHost, s));
  BCHAR_HIP(hipStreamSynchronize(s));
  double e = 0;
  for (int i = 0; i < nb; ++i) e = e > h[i] ? e : h[i];
  *max_col_err = e;
  ws.rewind(mk);
  return BCHAR_OK;
}

}  // namespace bchar
