// Memory helpers, prefix scans, stable bucket sort and reductions.
#include <list>

#include "device_util.hpp"
#include "internal.hpp"

namespace bchar {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

void DBuf::reserve(size_t n) {
  if (n <= bytes && p) return;
  if (p) {
    BCHAR_HIP(hipFree(p));
    p = nullptr;
    bytes = 0;
  }
  size_t want = n < 256 ? 256 : n;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    p = nullptr;
    throw Error{BCHAR_E_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(want) + " bytes failed"};
  }
  bytes = want;
}

void DBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

void* Arena::raw(size_t nbytes) {
  const size_t need = (nbytes + 255) & ~size_t(255);
  while (true) {
    if (cur < chunks.size()) {
      size_t o = (off + 255) & ~size_t(255);
      if (o + need <= chunks[cur].bytes) {
        off = o + need;
        return static_cast<char*>(chunks[cur].p) + o;
      }
      // does not fit: move on to the next chunk
      ++cur;
      off = 0;
      continue;
    }
    DBuf b;
    const size_t min_chunk = size_t(64) << 20;
    b.reserve(need > min_chunk ? need : min_chunk);
    chunks.push_back(b);
  }
}

void Arena::release() {
  for (auto& c : chunks) c.release();
  chunks.clear();
  reset();
}

// ---------------------------------------------------------------- scan

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void scan_tiles(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                           int32_t* __restrict__ tile_sums, int64_t n) {
  __shared__ int32_t sh[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t run = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t k = base + i;
    int32_t x = (k < n) ? in[k] : 0;
    v[i] = run;
    run += x;
  }
  // exclusive scan of per-thread totals across the block
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  int incl = wave_incl_scan_i(run);
  if (lane == kWave - 1) sh[w] = incl;
  __syncthreads();
  int woff = 0;
  for (int i = 0; i < w; ++i) woff += sh[i];
  int excl = woff + incl - run;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t k = base + i;
    if (k < n) out[k] = v[i] + excl;
  }
  if (threadIdx.x == kScanThreads - 1) tile_sums[blockIdx.x] = excl + run;
}

__global__ void scan_add(int32_t* __restrict__ out, const int32_t* __restrict__ tile_off,
                         int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
  const int32_t o = tile_off[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t kk = k + (int64_t)i * kScanThreads;
    if (kk < n) out[kk] += o;
  }
}

__global__ void write_total(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                            int64_t n) {
  // out[n] = out[n-1] + in[n-1]
  if (n > 0)
    out[n] = out[n - 1] + in[n - 1];
  else
    out[0] = 0;
}

// out[0..n) = exclusive scan of in, out[n] = total.  out must hold n+1.
void exclusive_scan_i32_async(const int32_t* in, int32_t* out, int64_t n, Arena& ws,
                              hipStream_t s) {
  if (n > 0) {
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    int32_t* sums = ws.get<int32_t>(tiles + 1);
    scan_tiles<<<(unsigned)tiles, kScanThreads, 0, s>>>(in, out, sums, n);
    BCHAR_HIP(hipGetLastError());
    if (tiles > 1) {
      int32_t* offs = ws.get<int32_t>(tiles + 1);
      exclusive_scan_i32_async(sums, offs, tiles, ws, s);
      scan_add<<<(unsigned)tiles, kScanThreads, 0, s>>>(out, offs, n);
      BCHAR_HIP(hipGetLastError());
    }
  }
  write_total<<<1, 1, 0, s>>>(in, out, n);
  BCHAR_HIP(hipGetLastError());
}

int64_t exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, Arena& ws,
                           hipStream_t s) {
  exclusive_scan_i32_async(in, out, n, ws, s);
  int32_t total = 0;
  BCHAR_HIP(hipMemcpyAsync(&total, out + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  BCHAR_HIP(hipStreamSynchronize(s));
  return total;
}

// ---------------------------------------------------------------- bucket sort

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_histogram(const int32_t* __restrict__ key, int64_t n,
                            int32_t* __restrict__ cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[key[i]], 1);
}

__global__ void k_scatter(const int32_t* __restrict__ key, int64_t n,
                          const int32_t* __restrict__ ptr, int32_t* __restrict__ fill,
                          int32_t* __restrict__ perm) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    int32_t k = key[i];
    int32_t slot = atomicAdd(&fill[k], 1);
    perm[ptr[k] + slot] = (int32_t)i;
  }
}

// The scatter above places items of a bucket in arbitrary order; sorting
// each (small) bucket by item id makes the result independent of timing.
__global__ void k_sort_buckets(const int32_t* __restrict__ ptr, int64_t nkeys,
                               int32_t* __restrict__ perm) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nkeys) return;
  const int32_t lo = ptr[b], hi = ptr[b + 1];
  for (int32_t i = lo + 1; i < hi; ++i) {
    int32_t v = perm[i];
    int32_t j = i - 1;
    while (j >= lo && perm[j] > v) {
      perm[j + 1] = perm[j];
      --j;
    }
    perm[j + 1] = v;
  }
}

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fill_i32<<<blocks_for(n, 256), 256, 0, s>>>(p, v, n);
  BCHAR_HIP(hipGetLastError());
}

__global__ void k_fill_f64(double* p, double v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fill_f64<<<blocks_for(n, 256), 256, 0, s>>>(p, v, n);
  BCHAR_HIP(hipGetLastError());
}

void bucket_sort(const int32_t* key, int64_t n, int64_t nkeys, int32_t* ptr, int32_t* perm,
                 Arena& ws, hipStream_t s) {
  Arena::Mark mark = ws.mark();
  int32_t* cnt = ws.get<int32_t>(nkeys + 1);
  fill_i32(cnt, 0, nkeys + 1, s);
  if (n > 0) {
    k_histogram<<<blocks_for(n, 256), 256, 0, s>>>(key, n, cnt);
    BCHAR_HIP(hipGetLastError());
  }
  exclusive_scan_i32_async(cnt, ptr, nkeys, ws, s);
  fill_i32(cnt, 0, nkeys + 1, s);
  if (n > 0) {
    k_scatter<<<blocks_for(n, 256), 256, 0, s>>>(key, n, ptr, cnt, perm);
    BCHAR_HIP(hipGetLastError());
    k_sort_buckets<<<blocks_for(nkeys, 256), 256, 0, s>>>(ptr, nkeys, perm);
    BCHAR_HIP(hipGetLastError());
  }
  ws.rewind(mark);
}

// ---------------------------------------------------------------- reductions

__global__ void k_max_abs(const double* __restrict__ v, int64_t n, double* __restrict__ part) {
  __shared__ double sh[16];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(v[i]));
  m = block_max(m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

double max_abs(const double* v, int64_t n, Arena& ws, hipStream_t s) {
  Arena::Mark mark = ws.mark();
  const int nb = 256;
  double* part = ws.get<double>(nb);
  k_max_abs<<<nb, 256, 0, s>>>(v, n, part);
  BCHAR_HIP(hipGetLastError());
  double h[nb];
  BCHAR_HIP(hipMemcpyAsync(h, part, sizeof(h), hipMemcpyDeviceToHost, s));
  BCHAR_HIP(hipStreamSynchronize(s));
  ws.rewind(mark);
  double m = 0;
  for (int i = 0; i < nb; ++i) m = m > h[i] ? m : h[i];
  return m;
}

}  // namespace bchar

// ---------------------------------------------------------------- kernel timing

#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <mutex>

namespace bchar {

bool trace_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("BCHAR_TRACE");
    return v && v[0] && v[0] != '0';
  }();
  return on;
}

double wall_seconds() {
  using clk = std::chrono::steady_clock;
  static const clk::time_point t0 = clk::now();
  return std::chrono::duration<double>(clk::now() - t0).count();
}

namespace {
struct ProfState {
  std::mutex mu;
  std::atomic<bool> on{false};  // a kernel is being timed (target non-empty)
  std::string target;     // kernel name being timed ("" = off)
  int64_t every = 1;      // time every `every`-th launch of it
  int64_t seen = 0;       // launches of it seen
  int64_t units = 0;      // replayable units seen
  // timed launches: start and end events, and whether the end has been
  // recorded (a scope records it when it closes); list nodes stay put, so a
  // scope keeps a pointer to its own
  struct Pair {
    hipEvent_t a, b;
    bool done;
    bool counted;   // false: opened before the last reset, dropped when drained
  };
  std::list<Pair> pending;
  std::vector<hipEvent_t> free_events;
  int64_t launches = 0;
  double total_ms = 0;
};
ProfState& prof() {
  static ProfState p;
  return p;
}
hipEvent_t take_event(ProfState& p) {
  if (!p.free_events.empty()) {
    hipEvent_t e = p.free_events.back();
    p.free_events.pop_back();
    return e;
  }
  hipEvent_t e;
  BCHAR_HIP(hipEventCreate(&e));
  return e;
}
// Sum the closed scopes (the caller holds the lock); each pair leaves the
// list as it is counted, so a failure part way counts nothing twice, and
// scopes still open are left for a later drain.
void drain(ProfState& p) {
  for (auto it = p.pending.begin(); it != p.pending.end();) {
    if (!it->done) {
      ++it;
      continue;
    }
    BCHAR_HIP(hipEventSynchronize(it->b));
    float ms = 0;
    BCHAR_HIP(hipEventElapsedTime(&ms, it->a, it->b));
    const hipEvent_t a = it->a, b = it->b;
    const bool counted = it->counted;
    it = p.pending.erase(it);
    if (counted) {
      p.total_ms += ms;
      p.launches += 1;
    }
    p.free_events.push_back(a);
    p.free_events.push_back(b);
  }
}
}  // namespace

thread_local ProfMode t_mode = ProfMode::normal;

void prof_set_mode(ProfMode m) { t_mode = m; }

bool prof_unit_due() {
  ProfState& p = prof();
  if (!p.on.load(std::memory_order_relaxed)) return false;
  std::lock_guard<std::mutex> g(p.mu);
  if (p.target.empty()) return false;
  return (p.units++ % p.every) == 0;
}

// The target is only read under the lock; a disabled scope costs one
// relaxed atomic load.
ProfScope::ProfScope(const char* name, hipStream_t st) : pair(nullptr), s(st) {
  ProfState& p = prof();
  if (t_mode == ProfMode::off || !p.on.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> g(p.mu);
  if (p.target != name) return;
  if (t_mode != ProfMode::all && (p.seen++ % p.every) != 0) return;
  hipEvent_t a = take_event(p), b = take_event(p);
  BCHAR_HIP(hipEventRecord(a, s));
  p.pending.push_back({a, b, false, true});
  pair = &p.pending.back();
}

// The end event is recorded under the lock and the pair marked closed in
// the same critical section, so that a concurrent drain never sees a pair
// whose end is not yet recorded.
ProfScope::~ProfScope() {
  if (!pair) return;
  ProfState& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  auto* pr = static_cast<ProfState::Pair*>(pair);
  (void)hipEventRecord(pr->b, s);
  pr->done = true;
}

}  // namespace bchar

extern "C" bchar_status bchar_profile_kernel_sampled(const char* name, int every) {
  if (every < 1) {
    bchar::set_error("every must be >= 1");
    return BCHAR_E_INVALID_ARG;
  }
  try {
    bchar::ProfState& p = bchar::prof();
    std::lock_guard<std::mutex> g(p.mu);
    bchar::drain(p);
    for (auto& pr : p.pending) pr.counted = false;   // scopes still open
    p.target = name ? name : "";
    p.on.store(!p.target.empty(), std::memory_order_relaxed);
    p.every = every;
    p.seen = 0;
    p.units = 0;
    p.launches = 0;
    p.total_ms = 0;
    return BCHAR_OK;
  } catch (const bchar::Error& e) {
    bchar::set_error(e.msg);
    return e.status;
  }
}

extern "C" bchar_status bchar_profile_kernel(const char* name) {
  return bchar_profile_kernel_sampled(name, 1);
}

extern "C" bchar_status bchar_profile_read(int64_t* launches, double* total_ms) {
  try {
    bchar::ProfState& p = bchar::prof();
    std::lock_guard<std::mutex> g(p.mu);
    bchar::drain(p);
    if (launches) *launches = p.launches;
    if (total_ms) *total_ms = p.total_ms;
    return BCHAR_OK;
  } catch (const bchar::Error& e) {
    bchar::set_error(e.msg);
    return e.status;
  }
}
