// The update (Sec. 2, eq. phys-inter-ELLAM) and the porous mass (Sec. 2.1).
//
// apply: c_out[K] = (sum_M A[K,M] c_in[M]) / |K|_phi.  Rows hold a few
//        entries (4-5 on the 3D workloads), so a group of 4 lanes takes a
//        row: the lanes stride the row's entries, combine with two xor
//        shuffles in a fixed order, and lane 0 writes.  Loads of A and of
//        the column indices are coalesced across the group; c_in is
//        gathered.
// mass:  sum_K phi_K |K| c_K with TwoSum-compensated per-thread sums,
//        a fixed-order block combine and a fixed-order final combine.
#include <mutex>

#include "device_util.hpp"
#include "internal.hpp"

namespace bchar {

constexpr int kRowLanes = 4;

__global__ void __launch_bounds__(256) k_apply(const int32_t* __restrict__ rptr,
                                               const int32_t* __restrict__ col,
                                               const double* __restrict__ a,
                                               const double* __restrict__ b,
                                               const double* __restrict__ cin, int64_t n,
                                               double* __restrict__ cout) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = g / kRowLanes;
  const int sub = (int)(g % kRowLanes);
  double acc = 0.0;
  if (i < n) {
    const int32_t lo = rptr[i], hi = rptr[i + 1];
    for (int32_t k = lo + sub; k < hi; k += kRowLanes) acc += a[k] * cin[col[k]];
  }
  acc += __shfl_xor(acc, 1, kWave);
  acc += __shfl_xor(acc, 2, kWave);
  if (i < n && sub == 0) cout[i] = acc / b[i];
}

void apply_transfer(const bchar_transfer_s* t, const double* cin, double* cout, hipStream_t s) {
  const bchar_mesh_s* m = t->mesh;
  const int64_t n = m->n_cells;
  {
    ::bchar::ProfScope ps_("k_apply", s);
    k_apply<<<blocks_for(n * kRowLanes, 256), 256, 0, s>>>(
        t->row_ptr.as<int32_t>(), t->col.as<int32_t>(), t->A.as<double>(), m->b.as<double>(), cin,
        n, cout);
  }
  BCHAR_HIP(hipGetLastError());
}

constexpr int kMassBlocks = 512;

// ghost (optional): cells left out (ghost cells hold boundary data)
__global__ void __launch_bounds__(256) k_mass_part(const double* __restrict__ b,
                                                   const double* __restrict__ c,
                                                   const uint8_t* __restrict__ ghost, int64_t n,
                                                   double* __restrict__ part) {
  __shared__ double sh[32];
  CSum acc;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    // phi_K |K| c_K as the product of two roundings; the sum is compensated
    if (!ghost || !ghost[i]) acc.add(b[i] * c[i]);
  }
  CSum tot = block_csum(acc, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = tot.hi;
    part[2 * blockIdx.x + 1] = tot.lo;
  }
}

// one wave: lane i combines the partials i, i + 64, ... in order, then a
// fixed butterfly (reproducible)
__global__ void k_mass_final(const double* __restrict__ part, int nparts,
                             double* __restrict__ out) {
  CSum acc;
  for (int i = threadIdx.x; i < nparts; i += kWave) {
    CSum o;
    o.hi = part[2 * i];
    o.lo = part[2 * i + 1];
    acc.add(o);
  }
  wave_csum(acc);
  if (threadIdx.x == 0) out[0] = acc.value();
}

double porous_mass(const bchar_mesh_s* m, const double* c, Arena& ws, hipStream_t s) {
  Arena::Mark mk = ws.mark();
  double* part = ws.get<double>(2 * kMassBlocks + 1);
  {
    ::bchar::ProfScope ps_("k_mass_part", s);
    k_mass_part<<<kMassBlocks, 256, 0, s>>>(m->b.as<double>(), c, m->ghost.as<uint8_t>(),
                                            m->n_cells, part);
  }
  BCHAR_HIP(hipGetLastError());
  {
    ::bchar::ProfScope ps_("k_mass_final", s);
    k_mass_final<<<1, 64, 0, s>>>(part, kMassBlocks, part + 2 * kMassBlocks);
  }
  BCHAR_HIP(hipGetLastError());
  double out = 0;
  BCHAR_HIP(hipMemcpyAsync(&out, part + 2 * kMassBlocks, sizeof(double), hipMemcpyDeviceToHost,
                           s));
  BCHAR_HIP(hipStreamSynchronize(s));
  ws.rewind(mk);
  return out;
}

// ---- the mass without allocation (bchar_mass_into)
//
// The block partials live in a file-scope device array, one copy per GPU
// for the life of the process.  Host code reaches it only through the
// address hipGetSymbolAddress returns on each device (the array's name is a
// host-side stand-in there), taken once per device on its first use.
constexpr int kMassScratch = 2 * kMassBlocks;   // hi and lo of every block partial
static __device__ __align__(256) double scratch[kMassScratch];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

static double* mass_scratch() {
  int dev = 0;
  BCHAR_HIP(hipGetDevice(&dev));
  BCHAR_REQUIRE(dev >= 0 && dev < kMaxDevices, BCHAR_E_UNSUPPORTED, "device index beyond 64");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    BCHAR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

void porous_mass_into(const bchar_mesh_s* m, const double* c, double* d_out, hipStream_t s) {
  // the same kernels and order as porous_mass: the same bits
  double* part = mass_scratch();
  {
    ::bchar::ProfScope ps_("k_mass_part", s);
    k_mass_part<<<kMassBlocks, 256, 0, s>>>(m->b.as<double>(), c, m->ghost.as<uint8_t>(),
                                            m->n_cells, part);
  }
  BCHAR_HIP(hipGetLastError());
  {
    ::bchar::ProfScope ps_("k_mass_final", s);
    k_mass_final<<<1, 64, 0, s>>>(part, kMassBlocks, d_out);
  }
  BCHAR_HIP(hipGetLastError());
}

}  // namespace bchar
