// sbr_api.hip -- the C-ABI of libsbr: handles, validation, host-side face
// grouping, buffer management and the order of kernel launches.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <optional>
#include <string>
#include <thread>
#include <vector>

#include "sbr_device.hpp"
#include "sbr_internal.hpp"

namespace sbr {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

namespace {
struct CachedBlock {
  void* p;
  size_t cap;
  hipStream_t s;
};
std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache;  // oldest first
size_t g_cache_bytes = 0;
constexpr size_t kCacheMax = size_t(8) << 30;       // cached bytes over all streams
constexpr size_t kCacheBlockMax = size_t(1) << 30;  // larger blocks are freed at once
// block size for a request: 1/16 steps of the power of two above it, at least 4 KiB
size_t block_size(size_t n) {
  if (n <= 4096) return 4096;
  size_t q = 4096;
  while (q < n) q <<= 1;
  const size_t g = std::max<size_t>(q / 16, 4096);
  return (n + g - 1) / g * g;
}
}  // namespace

void Buf::alloc(size_t n, hipStream_t s) {
  reset();
  const size_t want = block_size(n);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int best = -1;
    for (size_t i = 0; i < g_cache.size(); ++i) {
      const CachedBlock& b = g_cache[i];
      if (b.s == s && b.cap >= want && b.cap <= 2 * want && (best < 0 || b.cap < g_cache[best].cap)) best = (int)i;
    }
    if (best >= 0) {
      p = g_cache[best].p, cap = g_cache[best].cap;
      g_cache_bytes -= cap;
      g_cache.erase(g_cache.begin() + best);
      stream = s, bytes = n;
      return;
    }
  }
  hipError_t e = hipMallocAsync(&p, want, s);
  if (e != hipSuccess) {
    p = nullptr;
    set_error("device allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
    throw Error{SBR_E_OUT_OF_MEMORY};
  }
  stream = s, bytes = n, cap = want;
}

void Buf::reset() {
  if (p && cap > 0) {  // cap 0: a view, owned elsewhere
    if (cap > kCacheBlockMax) {
      (void)hipFreeAsync(p, stream);
    } else {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      g_cache.push_back(CachedBlock{p, cap, stream});
      g_cache_bytes += cap;
      while (g_cache_bytes > kCacheMax && !g_cache.empty()) {
        (void)hipFreeAsync(g_cache.front().p, g_cache.front().s);
        g_cache_bytes -= g_cache.front().cap;
        g_cache.erase(g_cache.begin());
      }
    }
  }
  p = nullptr;
  bytes = 0;
  cap = 0;
}

void buf_cache_flush(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (size_t i = 0; i < g_cache.size();) {
    if (g_cache[i].s == s) {
      (void)hipFreeAsync(g_cache[i].p, s);
      g_cache_bytes -= g_cache[i].cap;
      g_cache.erase(g_cache.begin() + i);
    } else {
      ++i;
    }
  }
}

thread_local Prof* g_prof = nullptr;

TimedLaunch::TimedLaunch(const char* n, hipStream_t st) : name(n), s(st) {
  if (g_prof && g_prof->wants(n)) {
    auto take = [](hipEvent_t* e) {
      if (!g_prof->spare.empty()) {
        *e = g_prof->spare.back();
        g_prof->spare.pop_back();
        return true;
      }
      return hipEventCreate(e) == hipSuccess;
    };
    if (take(&a) && take(&b)) {
      (void)hipEventRecord(a, s);
    } else {
      if (a) g_prof->spare.push_back(a);
      a = b = nullptr;
    }
  }
}
TimedLaunch::~TimedLaunch() {
  if (a && b && g_prof) {
    (void)hipEventRecord(b, s);
    g_prof->pending.push_back(Prof::Pending{name, a, b});
  }
}
static double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
void prof_add(const char* name, double ms) {
  if (!g_prof || !g_prof->enabled) return;
  for (auto& e : g_prof->acc)
    if (e.first == name) {
      e.second.first += ms;
      e.second.second += 1;
      return;
    }
  g_prof->acc.push_back({name, {ms, 1}});
}
HostPhase::HostPhase(const char* n) : name(n) {
  if (g_prof && g_prof->enabled && g_prof->only.empty()) t0 = now_ms();
}
HostPhase::~HostPhase() {
  if (g_prof && g_prof->enabled && g_prof->only.empty()) prof_add(name, now_ms() - t0);
}

void Prof::resolve() {
  for (auto& p : pending) {
    float ms = 0.0f;
    (void)hipEventSynchronize(p.b);
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    bool found = false;
    for (auto& e : acc)
      if (e.first == p.name) {
        e.second.first += ms;
        e.second.second += 1;
        found = true;
      }
    if (!found) acc.push_back({p.name, {(double)ms, 1}});
    spare.push_back(p.a);
    spare.push_back(p.b);
  }
  pending.clear();
}
void Prof::clear() {
  resolve();
  acc.clear();
}
void Prof::destroy_events() {
  resolve();
  for (hipEvent_t e : spare) (void)hipEventDestroy(e);
  spare.clear();
}

void retain(Handle* h) { h->refs.fetch_add(1); }
void release(Handle* h) {
  if (h && h->refs.fetch_sub(1) == 1) delete h;
}

void HostStage::reserve(size_t need) {
  if (bytes >= need) return;
  if (p) (void)hipHostFree(p);
  p = nullptr;
  bytes = 0;
  SBR_HIP(hipHostMalloc(&p, need, hipHostMallocDefault));
  bytes = need;
}
HostStage::~HostStage() {
  if (p) (void)hipHostFree(p);
  if (ev) (void)hipEventDestroy(ev);
}

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// run f, mapping exceptions to status codes
template <class F>
sbr_status guard(F&& f) {
  try {
    (void)hipGetLastError();  // a launch check must only see errors of this call
    f();
    return SBR_OK;
  } catch (const Error& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return SBR_E_OUT_OF_MEMORY;
  } catch (...) {
    set_error("unexpected internal error");
    return SBR_E_DEVICE;
  }
}

template <class H>
H* check_handle(void* p, int kind, const char* what) {
  SBR_CHECK(p != nullptr, SBR_E_INVALID_ARG, "%s handle is NULL", what);
  SBR_CHECK(static_cast<Handle*>(p)->kind == kind, SBR_E_INVALID_ARG, "%s handle has the wrong type", what);
  return static_cast<H*>(p);
}

// copy an input array to the host (it may be a device pointer)
template <class T>
std::vector<T> to_host(const T* p, size_t n, uint32_t flags, hipStream_t s) {
  std::vector<T> v(n);
  if (n == 0) return v;
  SBR_CHECK(p != nullptr, SBR_E_INVALID_ARG, "input array is NULL");
  if (flags & SBR_IN_DEVICE) {
    SBR_HIP(hipMemcpyAsync(v.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
  } else {
    std::memcpy(v.data(), p, n * sizeof(T));
  }
  return v;
}

// upload an input array into a library buffer (device-to-device when the input is on the device)
// Host sources are consumed before returning (the caller may free them at
// once); device sources are copied in stream order.
template <class T>
void upload(Buf& b, const T* p, size_t n, uint32_t flags, hipStream_t s) {
  b.alloc(n * sizeof(T), s);
  if (n == 0) return;
  SBR_CHECK(p != nullptr, SBR_E_INVALID_ARG, "input array is NULL");
  if (flags & SBR_IN_DEVICE) {
    SBR_HIP(hipMemcpyAsync(b.p, p, n * sizeof(T), hipMemcpyDeviceToDevice, s));
  } else {
    SBR_HIP(hipMemcpyAsync(b.p, p, n * sizeof(T), hipMemcpyHostToDevice, s));
    SBR_HIP(hipStreamSynchronize(s));
  }
}

// Host->device uploads of host-built arrays go through one pinned staging
// area owned by the context: each array is memcpy'd into it and copied
// asynchronously; the caller synchronises the stream before the staging area
// is written again.
struct Stager {
  HostStage* c;
  size_t off = 0;
  explicit Stager(HostStage& h) : c(&h) {}
  template <class T>
  void put(Buf& b, const T* src, size_t n, hipStream_t s) {
    b.alloc(n * sizeof(T), s);
    if (n == 0) return;
    const size_t bytes = n * sizeof(T);
    const size_t at = (off + 255) & ~size_t(255);
    if (at + bytes > c->bytes) {
      SBR_CHECK(off == 0, SBR_E_DEVICE, "staging area resized while in use");
      c->reserve(at + bytes + (1 << 20));
    }
    std::memcpy(static_cast<char*>(c->p) + at, src, bytes);
    SBR_HIP(hipMemcpyAsync(b.p, static_cast<char*>(c->p) + at, bytes, hipMemcpyHostToDevice, s));
    off = at + bytes;
  }
  // Packed uploads: add() places arrays side by side in the staging area,
  // flush() copies them with one transfer into `block` and points each Buf
  // at its part (views of `block`).  The staging area must already be large
  // enough (it is not resized here).
  struct Part {
    Buf* b;
    size_t at, bytes;
  };
  std::vector<Part> parts;
  template <class T>
  void add(Buf& b, const T* src, size_t n) {
    const size_t bytes = n * sizeof(T);
    const size_t at = (off + 255) & ~size_t(255);
    SBR_CHECK(at + bytes <= c->bytes, SBR_E_DEVICE, "staging area too small for packed uploads");
    if (bytes) std::memcpy(static_cast<char*>(c->p) + at, src, bytes);
    parts.push_back(Part{&b, at, bytes});
    off = at + bytes;
  }
  void flush(Buf& block, hipStream_t s) {
    if (parts.empty()) return;
    const size_t first = parts.front().at, total = std::max<size_t>(off - first, 1);
    block.alloc(total, s);
    SBR_HIP(hipMemcpyAsync(block.p, static_cast<char*>(c->p) + first, off - first, hipMemcpyHostToDevice, s));
    for (const Part& q : parts) q.b->view(block.as<char>() + (q.at - first), q.bytes);
    parts.clear();
  }
};

void set_device(sbr_context_s* c) {
  SBR_HIP(hipSetDevice(c->device));
  g_prof = &c->prof;
}

// triangle off + i of the FP32 array = triangle m(order ? order[i] : i), m =
// map or the identity: its vertices in the three cyclic axis orders (layout z
// holds axes z + 1, z + 2, z, so a ray whose dominant axis is z finds the
// coordinates of its shear frame in place), each vertex with one id in .w
__global__ void k_tri_gather(const uint32_t* __restrict__ order, const int32_t* __restrict__ map, int64_t n,
                             int64_t off, const float* __restrict__ v32, const int32_t* __restrict__ plane,
                             const int32_t* __restrict__ group, float4* __restrict__ tri) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t u = order ? order[i] : (uint32_t)i;
  const int32_t t = map ? map[u] : (int32_t)u;
  const float* v = v32 + 9 * (int64_t)t;
  const int64_t o = kTriVecs * (off + i);
  const float w[3] = {__int_as_float(t), __int_as_float(plane[t]), __int_as_float(group[t])};
  for (int z = 0; z < 3; ++z) {
    const int x = z == 2 ? 0 : z + 1, y = x == 2 ? 0 : x + 1;
    for (int j = 0; j < 3; ++j) tri[o + 3 * z + j] = make_float4(v[3 * j + x], v[3 * j + y], v[3 * j + z], w[j]);
  }
}

// Scene preparation on the device, so that the tree build starts before the
// host has the triangles.  Both kernels repeat the host's arithmetic
// operation for operation (the host computes the same centre and diagonal
// for its own steps): the FP64 box of all vertices, the centre 0.5 (lo + hi),
// vertices (float)(x - centre) and per-triangle FP32 boxes.  Rounding is
// monotone, so the FP32 scene bounds are (float)(lo - centre) and
// (float)(hi - centre).  Non-finite values (inputs the host then rejects)
// become 0 so that the tree build always sees finite boxes.
constexpr int kPrepBlocks = 64;
// worker threads (and streams) of a batched scene build
constexpr int kSceneWorkers = 8;
__global__ __launch_bounds__(256) void k_scene_bounds(const double* __restrict__ tri, int64_t nv,
                                                      double* __restrict__ part) {
  __shared__ double red[6][4];
  double b[6] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nv; v += (int64_t)gridDim.x * 256)
    for (int k = 0; k < 3; ++k) {
      const double x = tri[3 * v + k];
      b[k] = x < b[k] ? x : b[k];
      b[3 + k] = x > b[3 + k] ? x : b[3 + k];
    }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1)
    for (int k = 0; k < 6; ++k) {
      const double y = __shfl_xor(b[k], o, 64);
      b[k] = k < 3 ? (y < b[k] ? y : b[k]) : (y > b[k] ? y : b[k]);
    }
  if (lane == 0)
    for (int k = 0; k < 6; ++k) red[k][wv] = b[k];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    double r = red[k][0];
    for (int w = 1; w < 4; ++w) r = k < 3 ? (red[k][w] < r ? red[k][w] : r) : (red[k][w] > r ? red[k][w] : r);
    part[6 * blockIdx.x + k] = r;
  }
}
__device__ inline float finite_or_zero(float f) { return isfinite(f) ? f : 0.0f; }
__global__ __launch_bounds__(256) void k_scene_prep(const double* __restrict__ tri, int64_t T,
                                                    const double* __restrict__ part, int nb, float* __restrict__ v32,
                                                    float* __restrict__ blo, float* __restrict__ bhi,
                                                    float* __restrict__ bounds) {
  __shared__ double lh[6], cen[3];
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    double r = part[k];
    for (int j = 1; j < nb; ++j) {
      const double y = part[6 * j + k];
      r = k < 3 ? (y < r ? y : r) : (y > r ? y : r);
    }
    lh[k] = r;
  }
  __syncthreads();
  if (threadIdx.x < 3) cen[threadIdx.x] = 0.5 * (lh[threadIdx.x] + lh[3 + threadIdx.x]);
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < 6) {
    const int k = threadIdx.x;
    bounds[k] = finite_or_zero((float)(lh[k] - cen[k % 3]));
  }
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  float mn[3] = {1e30f, 1e30f, 1e30f}, mx[3] = {-1e30f, -1e30f, -1e30f};
  for (int v = 0; v < 3; ++v)
    for (int k = 0; k < 3; ++k) {
      const float f = finite_or_zero((float)(tri[9 * t + 3 * v + k] - cen[k]));
      v32[9 * t + 3 * v + k] = f;
      mn[k] = f < mn[k] ? f : mn[k], mx[k] = mx[k] < f ? f : mx[k];
    }
  for (int k = 0; k < 3; ++k) blo[3 * t + k] = mn[k], bhi[3 * t + k] = mx[k];
}

// hit chains by global ray id: thread = ray position, row = its global id
__global__ void k_hits_out(const int32_t* __restrict__ seq, int64_t NR, int K, RayOrder ord,
                           int32_t* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  const int64_t g = rid_of_pos(ord, r);
  bool ended = false;
  for (int k = 0; k <= K; ++k) {
    int32_t v = -2;
    if (!ended) {
      v = seq[(int64_t)k * NR + r];
      if (v < 0) ended = true;
    }
    out[g * (K + 1) + k] = v;
  }
}

// segments of one trace counted from its hit chains (traced entries per ray)
__global__ void k_count_segments(const int32_t* __restrict__ seq, int64_t NR, int K,
                                 unsigned long long* __restrict__ total) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long c = 0;
  if (r < NR) {
    for (int k = 0; k <= K; ++k) {
      ++c;
      if (seq[(int64_t)k * NR + r] < 0) break;
    }
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(total, c);
}

// Mean edge angle of the class-I geodesic of frequency N: a function of N
// alone (fixed-order FP64 sums), so one process-wide cache serves every
// context and thread.
std::mutex g_alpha_mu;
std::vector<std::pair<int, double>> g_alpha;
double alpha_for(sbr_context_s* c, int N) {
  {
    std::lock_guard<std::mutex> lk(g_alpha_mu);
    for (auto& pr : g_alpha)
      if (pr.first == N) return pr.second;
  }
  double mean = 0;
  geodesic_edge_stats(N, &mean, nullptr, nullptr, c->stream);
  std::lock_guard<std::mutex> lk(g_alpha_mu);
  for (auto& pr : g_alpha)
    if (pr.first == N) return pr.second;
  g_alpha.emplace_back(N, mean);
  return mean;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

// entry of the surrogate kernels: context check, device, profiler, error mapping
sbr_status nn_guard_call(sbr_context_t ctx, const std::function<void(hipStream_t)>& f) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    set_device(c);
    f(c->stream);
  });
}
}  // namespace sbr

using namespace sbr;

void* sbr_context_s::scratch_get(int slot, size_t bytes, hipStream_t s) {
  Buf& b = scratch[slot];
  if (b.p == nullptr || b.bytes < bytes || b.stream != s) b.alloc(bytes + bytes / 8, s);
  return b.p;
}

sbr_context_s::~sbr_context_s() {
  if (stream) (void)hipStreamSynchronize(stream);
  for (auto& b : scratch) b.reset();
  for (auto* g : graphs) delete g;
  if (stream) {
    buf_cache_flush(stream);
    (void)hipStreamSynchronize(stream);
  }
  for (SceneWorker* w : workers) {
    (void)hipStreamSynchronize(w->stream);
    buf_cache_flush(w->stream);
    (void)hipStreamSynchronize(w->stream);
    (void)hipStreamDestroy(w->stream);
    delete w;
  }
  prof.clear();
  prof.destroy_events();
  if (g_prof == &prof) g_prof = nullptr;
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}
sbr_scene_s::~sbr_scene_s() {
  if (ctx) (void)hipSetDevice(ctx->device);
  nodes.reset(), root_box.reset(), tri32.reset(), tri64.reset(), tplane.reset(), tgroup.reset(), tplaneid.reset();
  gplane.reset(), gmat.reset(), gstart.reset(), gtri.reset(), tables.reset(), wedges.reset();
  if (ctx) release(ctx);
}
sbr_trace_s::~sbr_trace_s() {
  if (ctx) (void)hipSetDevice(ctx->device);
  tx.reset(), seq.reset(), counters.reset(), work.reset();
  if (scene) release(scene);
  if (ctx) release(ctx);
}
sbr_diff_s::~sbr_diff_s() {
  if (ctx) (void)hipSetDevice(ctx->device);
  tx.reset(), rx.reset(), ids.reset(), rec.reset(), seg_start.reset(), power.reset();
  if (scene) release(scene);
  if (ctx) release(ctx);
}
sbr_scat_s::~sbr_scat_s() {
  if (ctx) (void)hipSetDevice(ctx->device);
  tx.reset(), rx.reset(), tiles.reset(), lobe.reset(), ids.reset(), rec.reset(), seg_start.reset(), power.reset();
  if (scene) release(scene);
  if (ctx) release(ctx);
}
sbr_paths_s::~sbr_paths_s() {
  if (ctx) (void)hipSetDevice(ctx->device);
  rx.reset(), key.reset(), geo.reset(), info.reset(), ang.reset(), power.reset(), seg_start.reset();
  ev_ray.reset(), ev_qk.reset();
  if (trace) release(trace);
  if (ctx) release(ctx);
}

extern "C" {

const char* sbr_last_error(void) { return g_err.c_str(); }
const char* sbr_version(void) { return "sbr-mi355x 0.1 (gfx950)"; }

void sbr_release(void* h) {
  if (!h) return;
  release(static_cast<Handle*>(h));
}

sbr_status sbr_context_create(int device, void* hip_stream, sbr_context_t* out) {
  return guard([&] {
    SBR_CHECK(out != nullptr, SBR_E_INVALID_ARG, "out is NULL");
    int ndev = 0;
    SBR_HIP(hipGetDeviceCount(&ndev));
    SBR_CHECK(device >= 0 && device < ndev, SBR_E_INVALID_ARG, "device %d of %d", device, ndev);
    SBR_HIP(hipSetDevice(device));
    // the allocation-free capacity's device array: its address on this device
    capacity_scratch_setup(device);
    auto* c = new sbr_context_s();
    c->device = device;
    if (hip_stream) {
      c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        delete c;
        SBR_HIP(e);
      }
      c->own_stream = true;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
      c->num_cus = cus;
    // keep freed stream-ordered memory cached in the pool between calls
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    *out = c;
  });
}

sbr_status sbr_synchronize(sbr_context_t ctx) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    set_device(c);
    SBR_HIP(hipStreamSynchronize(c->stream));
  });
}

// One scene built on stream s with staging area hs (the context's own, or a
// batch worker's); returns the scene once its build has finished on s.
static sbr_scene_s* scene_build_on(sbr_context_s* c, hipStream_t s, HostStage& hs, const double* tri_xyz, int64_t T,
                                   const float* eps_r, const float* sigma, const float* rough, uint32_t flags) {
  const bool dev_in = (flags & SBR_IN_DEVICE) != 0;
  // Scenes clustered with PLOC keep every triangle in the tree; they are
  // prepared on the device, so that the tree build starts at once and the
  // host's face grouping overlaps it.  Larger scenes (Morton-ordered LBVH
  // with a list of oversized triangles) are prepared on the host.
  const bool gpu_prep = T > 0 && T <= c->tune.bvh_ploc_max;
  // One pinned staging area serves the copies of device inputs (read
  // before the first upload) and the uploads; its size is set here, before
  // either is issued.
  const size_t bt = (size_t)T * 72, bm = (size_t)T * 4, o1 = (bt + 255) & ~size_t(255);
  const size_t o2 = o1 + ((bm + 255) & ~size_t(255)), o3 = o2 + ((bm + 255) & ~size_t(255));
  const size_t need = std::max(o3 + bm, (size_t)T * (72 + 32 + 8 + 32 + 16 + 4 + 4 + 60 + 4) + 4 + 20 * 256);
  hs.reserve(need);
  if (dev_in && gpu_prep && !hs.ev) SBR_HIP(hipEventCreateWithFlags(&hs.ev, hipEventDisableTiming));
  auto* sc = new sbr_scene_s();
  sc->ctx = c;
  retain(c);
  try {
    sc->T = T;
    std::vector<double> tri;
    std::vector<float> er, sg, rh;
    Stager st(hs);
    Buf dv32, dlo, dhi, order, dbvh_ids, dbig_ids, dpart, dbounds;
    uint32_t* depth_dev = nullptr;
    auto alloc_tree = [&] {
      sc->nodes.alloc((size_t)std::max<int64_t>(sc->n_bvh - 1, 1) * 64, s);
      sc->root_box.alloc(32, s);  // 6 floats of root box, then the depth word
      sc->tri32.alloc((size_t)T * kTriVecs * sizeof(float4), s);
      depth_dev = reinterpret_cast<uint32_t*>(sc->root_box.as<float>() + 6);
    };
    {
      HostPhase hp("host:scene_inputs");
      char* stg = static_cast<char*>(hs.p);
      if (dev_in && T > 0) {
        // device inputs: four copies into the staging area, then (device
        // preparation) an event the host waits for, or one synchronisation
        SBR_HIP(hipMemcpyAsync(stg, tri_xyz, bt, hipMemcpyDeviceToHost, s));
        SBR_HIP(hipMemcpyAsync(stg + o1, eps_r, bm, hipMemcpyDeviceToHost, s));
        SBR_HIP(hipMemcpyAsync(stg + o2, sigma, bm, hipMemcpyDeviceToHost, s));
        SBR_HIP(hipMemcpyAsync(stg + o3, rough, bm, hipMemcpyDeviceToHost, s));
        if (gpu_prep) SBR_HIP(hipEventRecord(hs.ev, s));
        else SBR_HIP(hipStreamSynchronize(s));
      } else if (T > 0) {
        tri.assign(tri_xyz, tri_xyz + (size_t)T * 9);
        er.assign(eps_r, eps_r + T), sg.assign(sigma, sigma + T), rh.assign(rough, rough + T);
      }
      if (gpu_prep) {
        if (dev_in) upload(sc->tri64, tri_xyz, (size_t)T * 9, flags, s);
        else st.put(sc->tri64, tri.data(), tri.size(), s);
        sc->n_big = 0;
        sc->n_bvh = T;
        alloc_tree();
        dv32.alloc((size_t)T * 36, s), dlo.alloc((size_t)T * 12, s), dhi.alloc((size_t)T * 12, s);
        dbounds.alloc(32, s), dpart.alloc((size_t)kPrepBlocks * 48, s), order.alloc((size_t)T * 4, s);
        const int nb = (int)std::min<int64_t>(kPrepBlocks, (3 * T + 255) / 256);
        hipLaunchKernelGGL(k_scene_bounds, dim3(nb), dim3(256), 0, s, sc->tri64.as<double>(), 3 * T,
                           dpart.as<double>());
        SBR_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_scene_prep, dim3(nblk(T, 256)), dim3(256), 0, s, sc->tri64.as<double>(), T,
                           dpart.as<double>(), nb, dv32.as<float>(), dlo.as<float>(), dhi.as<float>(),
                           dbounds.as<float>());
        SBR_LAUNCH_CHECK();
        BvhOut bo{sc->nodes.as<float4>(), order.as<uint32_t>(), sc->root_box.as<float>(), nullptr, depth_dev};
        bo.bounds_dev = dbounds.as<float>();
        build_bvh(dlo.as<float>(), dhi.as<float>(), T, nullptr, nullptr, bo, s, false);
        if (dev_in) SBR_HIP(hipEventSynchronize(hs.ev));
      }
      if (dev_in && T > 0) {
        tri.assign(reinterpret_cast<const double*>(stg), reinterpret_cast<const double*>(stg) + (size_t)T * 9);
        er.assign(reinterpret_cast<const float*>(stg + o1), reinterpret_cast<const float*>(stg + o1) + T);
        sg.assign(reinterpret_cast<const float*>(stg + o2), reinterpret_cast<const float*>(stg + o2) + T);
        rh.assign(reinterpret_cast<const float*>(stg + o3), reinterpret_cast<const float*>(stg + o3) + T);
      }
    }
    SBR_CHECK(finite_all(tri.data(), tri.size()), SBR_E_INVALID_ARG, "triangle coordinates must be finite");
    for (int64_t t = 0; t < T; ++t) {
      SBR_CHECK(std::isfinite(er[t]) && er[t] >= 1.0f, SBR_E_INVALID_ARG, "eps_r[%lld] = %g (needs >= 1)",
                (long long)t, er[t]);
      SBR_CHECK(std::isfinite(sg[t]) && sg[t] >= 0.0f, SBR_E_INVALID_ARG, "sigma[%lld] = %g", (long long)t,
                sg[t]);
      SBR_CHECK(std::isfinite(rh[t]) && rh[t] >= 0.0f, SBR_E_INVALID_ARG, "rough[%lld] = %g", (long long)t,
                rh[t]);
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t t = 0; t < T; ++t)
      for (int v = 0; v < 3; ++v)
        for (int k = 0; k < 3; ++k) {
          lo[k] = std::min(lo[k], tri[9 * t + 3 * v + k]);
          hi[k] = std::max(hi[k], tri[9 * t + 3 * v + k]);
        }
    if (T > 0) {
      for (int k = 0; k < 3; ++k) sc->center[k] = 0.5 * (lo[k] + hi[k]);
      sc->diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                           (hi[2] - lo[2]) * (hi[2] - lo[2]));
    }
    if (T == 0) {
      HostPhase hp("host:face_groups");
      face_groups({}, er.data(), sg.data(), rh.data(), sc->diag, sc->h_group, sc->h_plane, sc->n_groups,
                  sc->n_planes);
      sc->gstart.alloc(4, s);
      fill_u32(sc->gstart.as<uint32_t>(), 0, 1, s);
      SBR_HIP(hipStreamSynchronize(s));
      return sc;
    }
    if (!gpu_prep) {
      // ---- host preparation, uploaded first so that the GPU builds the
      // BVH while the host groups faces.
      // Scenes built with the Morton-ordered LBVH (above the context's
      // bvh_ploc_max triangles) keep oversized triangles (box diagonal above
      // a quarter of the scene's, at most kMaxBig, largest first) out of the
      // tree: there every ancestor of such a leaf gets a box as large as the
      // scene (a city's ground plane inflates a whole root-to-leaf chain),
      // so nearly every ray would descend those chains.  Every ray tests them
      // directly instead, before the traversal.  PLOC clustering merges
      // large boxes late, near the root, by itself, so smaller scenes keep
      // every triangle in the tree.
      constexpr int kMaxBig = 16;
      std::vector<std::pair<double, int32_t>> cand;
      for (int64_t t = 0; t < T; ++t) {
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
          const double a = tri[9 * t + k], b = tri[9 * t + 3 + k], cc = tri[9 * t + 6 + k];
          const double e = std::max(a, std::max(b, cc)) - std::min(a, std::min(b, cc));
          d2 += e * e;
        }
        if (d2 > 0.0625 * sc->diag * sc->diag) cand.push_back({d2, (int32_t)t});
      }
      std::sort(cand.begin(), cand.end(), [](const auto& x, const auto& y) {
        return x.first > y.first || (x.first == y.first && x.second < y.second);
      });
      if (cand.size() > (size_t)kMaxBig) cand.resize(kMaxBig);
      std::vector<int32_t> big_ids;
      std::vector<char> is_big((size_t)T, 0);
      for (const auto& cb : cand) big_ids.push_back(cb.second), is_big[cb.second] = 1;
      std::sort(big_ids.begin(), big_ids.end());
      std::vector<int32_t> bvh_ids;
      for (int64_t t = 0; t < T; ++t)
        if (!is_big[t]) bvh_ids.push_back((int32_t)t);
      sc->n_big = (int)big_ids.size();
      sc->n_bvh = (int64_t)bvh_ids.size();
      // FP32 vertices centred on the scene box; boxes of the tree's
      // triangles (rounded outward in the builder)
      std::vector<float> v32((size_t)T * 9), blo((size_t)sc->n_bvh * 3), bhi((size_t)sc->n_bvh * 3);
      float slo[3] = {1e30f, 1e30f, 1e30f}, shi[3] = {-1e30f, -1e30f, -1e30f};
      for (int64_t t = 0; t < T; ++t)
        for (int k = 0; k < 3; ++k)
          for (int v = 0; v < 3; ++v) v32[9 * t + 3 * v + k] = (float)(tri[9 * t + 3 * v + k] - sc->center[k]);
      for (int64_t j = 0; j < sc->n_bvh; ++j) {
        const int64_t t = bvh_ids[j];
        for (int k = 0; k < 3; ++k) {
          float mn = 1e30f, mx = -1e30f;
          for (int v = 0; v < 3; ++v)
            mn = std::min(mn, v32[9 * t + 3 * v + k]), mx = std::max(mx, v32[9 * t + 3 * v + k]);
          blo[3 * j + k] = mn, bhi[3 * j + k] = mx;
          slo[k] = std::min(slo[k], mn), shi[k] = std::max(shi[k], mx);
        }
      }
      {
        HostPhase hp_up("host:scene_upload");
        st.put(dv32, v32.data(), v32.size(), s);
        st.put(dlo, blo.data(), blo.size(), s);
        st.put(dhi, bhi.data(), bhi.size(), s);
        st.put(dbvh_ids, bvh_ids.data(), bvh_ids.size(), s);
        st.put(dbig_ids, big_ids.data(), big_ids.size(), s);
      }
      alloc_tree();
      if (sc->n_bvh > 0) {
        order.alloc((size_t)sc->n_bvh * 4, s);
        build_bvh(dlo.as<float>(), dhi.as<float>(), sc->n_bvh, slo, shi,
                  BvhOut{sc->nodes.as<float4>(), order.as<uint32_t>(), sc->root_box.as<float>(), nullptr, depth_dev},
                  s, /*linear=*/true);
      }
    }
    // ---- planes, face groups and group tables on the host (overlapping the build)
    std::vector<Plane> pl((size_t)T);
    for (int64_t t = 0; t < T; ++t) {
      const d3 a = ld3(&tri[9 * t]), b = ld3(&tri[9 * t + 3]), cc = ld3(&tri[9 * t + 6]);
      const d3 nn = cross(b - a, cc - a);
      const double area2 = norm(nn);
      SBR_CHECK(0.5 * area2 > 1e-12 * sc->diag * sc->diag, SBR_E_INVALID_ARG,
                "triangle %lld is degenerate (area %g)", (long long)t, 0.5 * area2);
      const d3 n = nn * (1.0 / area2);
      pl[t] = Plane{{n.x, n.y, n.z}, dot(n, a)};
    }
    {
      HostPhase hp("host:face_groups");
      face_groups(pl, er.data(), sg.data(), rh.data(), sc->diag, sc->h_group, sc->h_plane, sc->n_groups,
                  sc->n_planes);
    }
    // per-triangle FP64 planes, per-group plane/material/members
    std::vector<double4> tpl((size_t)T);
    for (int64_t t = 0; t < T; ++t) tpl[t] = make_double4(pl[t].n[0], pl[t].n[1], pl[t].n[2], pl[t].c);
    const int G = sc->n_groups;
    std::vector<int32_t> gfirst(G, -1), gstart(G + 1, 0), gtri((size_t)T), fill(G, 0);
    for (int64_t t = 0; t < T; ++t) {
      const int g = sc->h_group[t];
      if (gfirst[g] < 0) gfirst[g] = (int)t;
      gstart[g + 1]++;
    }
    for (int g = 0; g < G; ++g) gstart[g + 1] += gstart[g];
    for (int64_t t = 0; t < T; ++t) {
      const int g = sc->h_group[t];
      gtri[gstart[g] + fill[g]++] = (int)t;
    }
    std::vector<double4> gpl(G);
    std::vector<float4> gmt(G);
    for (int g = 0; g < G; ++g) {
      gpl[g] = tpl[gfirst[g]];
      gmt[g] = make_float4(er[gfirst[g]], sg[gfirst[g]], rh[gfirst[g]], 0.0f);
    }
    {
      HostPhase hp_up("host:scene_upload");
      if (!gpu_prep) st.put(sc->tri64, tri.data(), tri.size(), s);
      st.add(sc->tplane, tpl.data(), tpl.size());
      st.add(sc->tgroup, sc->h_group.data(), sc->h_group.size());
      st.add(sc->tplaneid, sc->h_plane.data(), sc->h_plane.size());
      st.add(sc->gplane, gpl.data(), gpl.size());
      st.add(sc->gmat, gmt.data(), gmt.size());
      st.add(sc->gstart, gstart.data(), gstart.size());
      st.add(sc->gtri, gtri.data(), gtri.size());
      st.flush(sc->tables, s);
    }
    if (sc->n_bvh > 0) {
      // leaves in tree order; device-prepared scenes hold every triangle in the tree
      hipLaunchKernelGGL(k_tri_gather, dim3(nblk(sc->n_bvh, 256)), dim3(256), 0, s, order.as<uint32_t>(),
                         gpu_prep ? (const int32_t*)nullptr : dbvh_ids.as<int32_t>(), sc->n_bvh, (int64_t)0,
                         dv32.as<float>(), sc->tplaneid.as<int32_t>(), sc->tgroup.as<int32_t>(),
                         sc->tri32.as<float4>());
      SBR_LAUNCH_CHECK();
    }
    if (sc->n_big > 0) {
      hipLaunchKernelGGL(k_tri_gather, dim3(1), dim3(64), 0, s, (const uint32_t*)nullptr, dbig_ids.as<int32_t>(),
                         (int64_t)sc->n_big, sc->n_bvh, dv32.as<float>(), sc->tplaneid.as<int32_t>(),
                         sc->tgroup.as<int32_t>(), sc->tri32.as<float4>());
      SBR_LAUNCH_CHECK();
    }
    // one synchronisation: root box and depth of the tree; it also frees the staging area
    sc->bvh_depth = 1;
    if (sc->n_bvh > 0) {
      float rb[7];
      SBR_HIP(hipMemcpyAsync(rb, sc->root_box.p, sizeof rb, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
      for (int k = 0; k < 6; ++k) sc->root_host[k] = rb[k];
      uint32_t depth;
      std::memcpy(&depth, &rb[6], 4);
      SBR_CHECK(depth != 0xffffffffu, SBR_E_DEVICE, "BVH clustering did not reach a single root");
      sc->bvh_depth = (int)depth;
      SBR_CHECK(sc->bvh_depth <= 64, SBR_E_UNSUPPORTED, "BVH depth %d exceeds the traversal stack",
                sc->bvh_depth);
    } else {
      SBR_HIP(hipStreamSynchronize(s));
    }
  } catch (...) {
    // copies from the staging area and the tree build may still be in
    // flight: let them finish before the scene and the staging area go
    (void)hipStreamSynchronize(s);
    release(sc);
    throw;
  }
  return sc;
}

sbr_status sbr_scene_build(sbr_context_t ctx, const double* tri_xyz, int64_t T, const float* eps_r,
                           const float* sigma, const float* rough, uint32_t flags, sbr_scene_t* out) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    SBR_CHECK(out != nullptr, SBR_E_INVALID_ARG, "out is NULL");
    SBR_CHECK(T >= 0 && T < (int64_t(1) << 30), SBR_E_INVALID_ARG, "triangle count %lld", (long long)T);
    if (T > 0) SBR_CHECK(tri_xyz && eps_r && sigma && rough, SBR_E_INVALID_ARG, "input array is NULL");
    set_device(c);
    HostPhase hp_all("host:scene_build");
    *out = scene_build_on(c, c->stream, c->stage, tri_xyz, T, eps_r, sigma, rough, flags);
  });
}

sbr_status sbr_scene_build_batch(sbr_context_t ctx, int32_t n, const double* const* tri_xyz, const int64_t* T,
                                 const float* const* eps_r, const float* const* sigma, const float* const* rough,
                                 uint32_t flags, sbr_scene_t* out) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    SBR_CHECK(n >= 1 && tri_xyz && T && eps_r && sigma && rough && out, SBR_E_INVALID_ARG, "batch arguments");
    for (int i = 0; i < n; ++i) {
      SBR_CHECK(T[i] >= 0 && T[i] < (int64_t(1) << 30), SBR_E_INVALID_ARG, "triangle count %lld of scene %d",
                (long long)T[i], i);
      if (T[i] > 0)
        SBR_CHECK(tri_xyz[i] && eps_r[i] && sigma[i] && rough[i], SBR_E_INVALID_ARG, "input array of scene %d is NULL",
                  i);
    }
    set_device(c);
    HostPhase hp_all("host:scene_build");
    // device inputs may have been written by earlier work on the context's
    // stream; the workers' streams read them only after it
    if (flags & SBR_IN_DEVICE) SBR_HIP(hipStreamSynchronize(c->stream));
    const int nw = std::min(n, kSceneWorkers);
    while ((int)c->workers.size() < nw) {
      auto* w = new SceneWorker();
      const hipError_t e = hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        delete w;
        SBR_HIP(e);
      }
      c->workers.push_back(w);
    }
    // Workers take scenes from a shared counter, largest first (the build
    // time grows with the triangle count, so the big scenes start early and
    // the small ones fill in); each builds on its own stream and staging
    // area.  Profiling stays with the calling thread (the workers record no
    // events).  A failure stops the others after their current scene; its
    // message names the scene.
    std::vector<int> by_size((size_t)n);
    for (int i = 0; i < n; ++i) by_size[i] = i;
    std::stable_sort(by_size.begin(), by_size.end(), [&](int a, int b) { return T[a] > T[b]; });
    std::vector<sbr_scene_s*> res((size_t)n, nullptr);
    std::atomic<int> next{0};
    std::atomic<bool> failed{false};
    std::mutex err_mu;
    sbr_status err_st = SBR_OK;
    std::string err_text;
    auto work = [&](int w) {
      int i = -1;
      try {
        SBR_HIP(hipSetDevice(c->device));
        SceneWorker& wk = *c->workers[w];
        for (int k; !failed.load() && (k = next.fetch_add(1)) < n;) {
          i = by_size[k];
          res[i] = scene_build_on(c, wk.stream, wk.stage, tri_xyz[i], T[i], eps_r[i], sigma[i], rough[i], flags);
          res[i]->rehome(c->stream);
        }
      } catch (const Error& e) {
        std::lock_guard<std::mutex> lk(err_mu);
        if (!failed.exchange(true)) err_st = e.st, err_text = "scene " + std::to_string(i) + ": " + g_err;
      } catch (...) {
        std::lock_guard<std::mutex> lk(err_mu);
        if (!failed.exchange(true)) err_st = SBR_E_DEVICE, err_text = "unexpected internal error in a scene build";
      }
    };
    std::vector<std::thread> th;
    for (int w = 0; w < nw; ++w) th.emplace_back(work, w);
    for (auto& t : th) t.join();
    if (failed.load()) {
      for (sbr_scene_s* sc : res)
        if (sc) release(sc);
      set_error("%s", err_text.c_str());
      throw Error{err_st};
    }
    for (int i = 0; i < n; ++i) out[i] = res[i];
  });
}

sbr_status sbr_scene_info(sbr_scene_t s, int32_t* n_groups, int32_t* n_planes, int32_t* bvh_depth) {
  return guard([&] {
    auto* sc = check_handle<sbr_scene_s>(s, kScene, "scene");
    if (n_groups) *n_groups = sc->n_groups;
    if (n_planes) *n_planes = sc->n_planes;
    if (bvh_depth) *bvh_depth = sc->bvh_depth;
  });
}

sbr_status sbr_scene_groups(sbr_scene_t s, int32_t* group, int32_t* plane) {
  return guard([&] {
    auto* sc = check_handle<sbr_scene_s>(s, kScene, "scene");
    if (group) std::copy(sc->h_group.begin(), sc->h_group.end(), group);
    if (plane) std::copy(sc->h_plane.begin(), sc->h_plane.end(), plane);
  });
}

sbr_status sbr_trace(sbr_context_t ctx, sbr_scene_t scene, const double* tx_xyz, int32_t Nt, int32_t N,
                     int32_t K, uint32_t flags, sbr_trace_t* out) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    auto* sc = check_handle<sbr_scene_s>(scene, kScene, "scene");
    SBR_CHECK(out != nullptr, SBR_E_INVALID_ARG, "out is NULL");
    SBR_CHECK(Nt >= 1, SBR_E_INVALID_ARG, "Nt = %d", Nt);
    SBR_CHECK(N >= 1 && N <= 46340, SBR_E_INVALID_ARG, "geodesic_N = %d", N);
    SBR_CHECK(K >= 0 && K <= SBR_MAX_BOUNCES, SBR_E_INVALID_ARG, "max_bounces = %d", K);
    const int64_t R = 10LL * N * N + 2;
    SBR_CHECK((int64_t)Nt * R < (int64_t(1) << 32) - (int64_t(1) << 22), SBR_E_UNSUPPORTED,
              "Nt * rays = %lld exceeds 2^32 - 2^22",
              (long long)Nt * R);
    set_device(c);
    hipStream_t s = c->stream;
    std::optional<HostPhase> hp_step;
    hp_step.emplace("host:trace_setup");
    const auto htx = to_host(tx_xyz, (size_t)Nt * 3, flags, s);
    SBR_CHECK(finite_all(htx.data(), htx.size()), SBR_E_INVALID_ARG, "tx coordinates must be finite");
    auto* tr = new sbr_trace_s();
    tr->ctx = c, tr->scene = sc;
    retain(c), retain(sc);
    try {
      tr->Nt = Nt, tr->N = N, tr->K = K, tr->R = R, tr->NR = (int64_t)Nt * R;
      tr->emin = Nt > 1 && c->tune.trace_order == 1;
      tr->h_tx = htx;
      // a device-resident input is copied on the device (no second host round trip)
      if (flags & SBR_IN_DEVICE) upload(tr->tx, tx_xyz, tr->h_tx.size(), flags, s);
      else upload(tr->tx, tr->h_tx.data(), tr->h_tx.size(), 0, s);
      tr->seq.alloc((size_t)(K + 1) * tr->NR * 4, s);
      tr->counters.alloc((size_t)trace_counter_words(K) * 4, s);
      void* ra = c->scratch_get(0, trace_ray_bytes(tr->NR), s);
      void* rb = K > 0 ? c->scratch_get(1, trace_ray_bytes(tr->NR), s) : ra;
      TraceLaunch L{};
      L.ctx = c;
      L.scene = sc, L.tx = tr->tx.as<double>(), L.Nt = Nt, L.N = N, L.K = K, L.R = R, L.NR = tr->NR;
      L.emin = tr->emin;
      L.seq = tr->seq.as<int32_t>();
      L.counters = tr->counters.as<uint32_t>();
      L.work = nullptr;
      if (c->count_work) {
        tr->work.alloc(16, s);
        fill_u32(tr->work.as<uint32_t>(), 0, 4, s);
        L.work = tr->work.as<unsigned long long>();
        tr->counted = true;
      }
      L.block = 256;
      L.grid = c->num_cus * c->tune.trace_blocks_per_cu;
      L.chunk = c->tune.trace_chunk;
      L.leaf_share = c->tune.trace_leaf_share;
      L.packet = c->tune.trace_packet;
      hp_step.emplace("host:trace_launch");
      launch_trace(L, ra, rb, s);
    } catch (...) {
      release(tr);
      throw;
    }
    *out = tr;
  });
}

sbr_status sbr_trace_batch(sbr_context_t ctx, int32_t n, const sbr_scene_t* scenes, const double* const* tx_xyz,
                           const int32_t* Nt, const int32_t* Nv, const int32_t* Kv, uint32_t flags,
                           sbr_trace_t* out) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    SBR_CHECK(n >= 1 && scenes && tx_xyz && Nt && Nv && Kv && out, SBR_E_INVALID_ARG, "batch arguments");
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
      check_handle<sbr_scene_s>(scenes[i], kScene, "scene");
      SBR_CHECK(Nt[i] >= 1, SBR_E_INVALID_ARG, "Nt[%d] = %d", i, Nt[i]);
      SBR_CHECK(Nv[i] >= 1 && Nv[i] <= 46340, SBR_E_INVALID_ARG, "geodesic_N[%d] = %d", i, Nv[i]);
      SBR_CHECK(Kv[i] >= 0 && Kv[i] <= SBR_MAX_BOUNCES, SBR_E_INVALID_ARG, "max_bounces[%d] = %d", i, Kv[i]);
      total += (int64_t)Nt[i] * (10LL * Nv[i] * Nv[i] + 2);
    }
    SBR_CHECK(total < (int64_t(1) << 32) - (int64_t(1) << 22), SBR_E_UNSUPPORTED, "batch of %lld rays", (long long)total);
    set_device(c);
    hipStream_t s = c->stream;
    std::vector<sbr_trace_s*> trs;
    try {
      for (int i = 0; i < n; ++i) {
        auto* sc = static_cast<sbr_scene_s*>(scenes[i]);
        const auto htx = to_host(tx_xyz[i], (size_t)Nt[i] * 3, flags, s);
        SBR_CHECK(finite_all(htx.data(), htx.size()), SBR_E_INVALID_ARG, "tx[%d] coordinates must be finite", i);
        auto* tr = new sbr_trace_s();
        tr->ctx = c, tr->scene = sc;
        retain(c), retain(sc);
        trs.push_back(tr);
        tr->Nt = Nt[i], tr->N = Nv[i], tr->K = Kv[i], tr->R = 10LL * Nv[i] * Nv[i] + 2;
        tr->NR = (int64_t)Nt[i] * tr->R;
        tr->emin = Nt[i] > 1 && c->tune.trace_order == 1;
        tr->h_tx = htx;
        tr->batched = true;
        tr->seq.alloc((size_t)(tr->K + 1) * tr->NR * 4, s);
        tr->counters.alloc(4, s);
      }
      {
        size_t need = 0;
        for (auto* tr : trs) need += tr->h_tx.size() * 8 + 256;
        c->stage.reserve(need);
      }
      Stager st(c->stage);
      for (auto* tr : trs) st.put(tr->tx, tr->h_tx.data(), tr->h_tx.size(), s);
      int Kmax = 0;
      for (auto* tr : trs) Kmax = std::max(Kmax, tr->K);
      void* ra = c->scratch_get(0, trace_ray_bytes(total), s);
      void* rb = c->scratch_get(1, trace_ray_bytes(total), s);
      Buf cnt, stamps;
      cnt.alloc((size_t)trace_counter_words(Kmax) * 4, s);
      stamps.alloc((size_t)2 * n * 8, s);
      unsigned long long* t_first = stamps.as<unsigned long long>();
      launch_trace_batch(trs, c->num_cus * c->tune.trace_blocks_per_cu, c->tune.trace_chunk,
                         c->tune.trace_leaf_share, ra, rb, cnt.as<uint32_t>(), t_first, t_first + n, s);
      std::vector<unsigned long long> h(2 * (size_t)n);
      SBR_HIP(hipMemcpyAsync(h.data(), stamps.p, h.size() * 8, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
      int khz = 100000;
      (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device);
      for (int i = 0; i < n; ++i)
        trs[i]->latency_ms = h[n + i] >= h[i] ? (double)(h[n + i] - h[i]) / (double)khz : 0.0;
    } catch (...) {
      for (auto* tr : trs) release(tr);
      throw;
    }
    for (int i = 0; i < n; ++i) out[i] = trs[i];
  });
}

sbr_status sbr_trace_latency(sbr_trace_t t, double* ms) {
  return guard([&] {
    auto* tr = check_handle<sbr_trace_s>(t, kTrace, "trace");
    SBR_CHECK(ms != nullptr, SBR_E_INVALID_ARG, "ms is NULL");
    *ms = tr->latency_ms;
  });
}

sbr_status sbr_trace_info(sbr_trace_t t, int64_t* rays, int64_t* segments) {
  return guard([&] {
    auto* tr = check_handle<sbr_trace_s>(t, kTrace, "trace");
    set_device(tr->ctx);
    if (tr->segments < 0 && tr->batched) {
      hipStream_t s = tr->ctx->stream;
      Buf cnt;
      cnt.alloc(8, s);
      fill_u32(cnt.as<uint32_t>(), 0, 2, s);
      { TimedLaunch tl_("misc", s); hipLaunchKernelGGL(k_count_segments, dim3(nblk(tr->NR, 256)), dim3(256), 0, s, tr->seq.as<int32_t>(), tr->NR, tr->K, cnt.as<unsigned long long>()); }
      SBR_LAUNCH_CHECK();
      unsigned long long v = 0;
      SBR_HIP(hipMemcpyAsync(&v, cnt.p, 8, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
      tr->segments = (int64_t)v;
    }
    if (tr->segments < 0) {
      std::vector<uint32_t> cnt((size_t)trace_counter_words(tr->K));
      SBR_HIP(hipMemcpyAsync(cnt.data(), tr->counters.p, cnt.size() * 4, hipMemcpyDeviceToHost, tr->ctx->stream));
      SBR_HIP(hipStreamSynchronize(tr->ctx->stream));
      int64_t seg = tr->NR;  // survivors of bounce k are the rays of bounce k + 1
      for (int k = 0; k < tr->K; ++k)
        for (int x = 0; x < 8; ++x) seg += cnt[(size_t)kCtrWords * k + kCtrOut + 32 * x];
      tr->segments = seg;
    }
    if (rays) *rays = tr->NR;
    if (segments) *segments = tr->segments;
  });
}

sbr_status sbr_trace_hits(sbr_trace_t t, int32_t* seq, float* uv, uint32_t flags) {
  return guard([&] {
    auto* tr = check_handle<sbr_trace_s>(t, kTrace, "trace");
    SBR_CHECK(seq != nullptr || uv != nullptr, SBR_E_INVALID_ARG, "seq and uv are NULL");
    set_device(tr->ctx);
    hipStream_t s = tr->ctx->stream;
    const size_t n = (size_t)tr->NR * (tr->K + 1);
    const bool dev = flags & SBR_OUT_DEVICE;
    Buf tmp, tmp_uv;
    if (seq) {
      int32_t* dst = seq;
      if (!dev) tmp.alloc(n * 4, s), dst = tmp.as<int32_t>();
      { ::sbr::TimedLaunch tl_("misc", s); hipLaunchKernelGGL(k_hits_out, dim3(nblk(tr->NR, 256)), dim3(256), 0, s, tr->seq.as<int32_t>(), tr->NR, tr->K,
                         RayOrder{tr->R, (int32_t)tr->Nt, (int32_t)tr->emin}, dst); }
      SBR_LAUNCH_CHECK();
      if (!dev) SBR_HIP(hipMemcpyAsync(seq, dst, n * 4, hipMemcpyDeviceToHost, s));
    }
    if (uv) {
      float* dst = uv;
      if (!dev) tmp_uv.alloc(n * 8, s), dst = tmp_uv.as<float>();
      run_hits_uv(tr, dst, s);
      if (!dev) SBR_HIP(hipMemcpyAsync(uv, dst, n * 8, hipMemcpyDeviceToHost, s));
    }
    if (!dev) SBR_HIP(hipStreamSynchronize(s));
  });
}

sbr_status sbr_receive(sbr_context_t ctx, sbr_trace_t t, const double* rx_xyz, int32_t Nr, double alpha_rad,
                       double radius_coeff, uint32_t flags, sbr_paths_t* out) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    auto* tr = check_handle<sbr_trace_s>(t, kTrace, "trace");
    SBR_CHECK(out != nullptr, SBR_E_INVALID_ARG, "out is NULL");
    SBR_CHECK(Nr >= 1 && (int64_t)Nr < (int64_t(1) << 26), SBR_E_INVALID_ARG, "Nr = %d", Nr);
    SBR_CHECK((int64_t)Nr * tr->Nt < (int64_t(1) << 31), SBR_E_UNSUPPORTED, "Nr * Nt too large");
    SBR_CHECK(std::isfinite(radius_coeff) && radius_coeff > 0, SBR_E_INVALID_ARG, "radius_coeff = %g",
              radius_coeff);
    SBR_CHECK(std::isfinite(alpha_rad), SBR_E_INVALID_ARG, "alpha must be finite");
    set_device(c);
    hipStream_t s = c->stream;
    // Up to kLbvhSmall receivers are prepared and checked on the device (a
    // host copy of device-resident points would wait for the trace queued
    // before it); larger sets go through the host.
    const bool dev_prep = Nr <= kLbvhSmall;
    SBR_CHECK(rx_xyz != nullptr, SBR_E_INVALID_ARG, "rx is NULL");
    std::vector<double> hrx;
    if (!dev_prep) {
      hrx = to_host(rx_xyz, (size_t)Nr * 3, flags, s);
      SBR_CHECK(finite_all(hrx.data(), hrx.size()), SBR_E_INVALID_ARG, "rx coordinates must be finite");
      for (int q = 0; q < Nr; ++q)
        for (int p = 0; p < tr->Nt; ++p)
          SBR_CHECK(!(hrx[3 * q] == tr->h_tx[3 * p] && hrx[3 * q + 1] == tr->h_tx[3 * p + 1] &&
                      hrx[3 * q + 2] == tr->h_tx[3 * p + 2]),
                    SBR_E_INVALID_ARG, "rx %d coincides with tx %d", q, p);
    }
    auto* ps = new sbr_paths_s();
    ps->ctx = c, ps->trace = tr;
    retain(c), retain(tr);
    try {
      ps->Nr = Nr;
      ps->coeff = radius_coeff;
      ps->alpha = alpha_rad > 0 ? alpha_rad : alpha_for(c, tr->N);
      if (flags & SBR_IN_DEVICE) upload(ps->rx, rx_xyz, (size_t)Nr * 3, flags, s);
      else upload(ps->rx, rx_xyz, (size_t)Nr * 3, 0, s);
      run_receive(ps, dev_prep ? nullptr : hrx.data(), s);
    } catch (...) {
      release(ps);
      throw;
    }
    *out = ps;
  });
}

sbr_status sbr_paths_info(sbr_paths_t p, int64_t* events, int64_t* keys, int64_t* paths) {
  return guard([&] {
    auto* ps = check_handle<sbr_paths_s>(p, kPaths, "paths");
    if (events) *events = ps->n_events;
    if (keys) *keys = ps->n_keys;
    if (paths) *paths = ps->n_paths;
  });
}

sbr_status sbr_paths_count(sbr_paths_t p, int64_t* n) {
  return guard([&] {
    auto* ps = check_handle<sbr_paths_s>(p, kPaths, "paths");
    SBR_CHECK(n != nullptr, SBR_E_INVALID_ARG, "n is NULL");
    *n = ps->n_paths;
  });
}

sbr_status sbr_paths_events(sbr_paths_t p, int64_t capacity, uint32_t* ray, int32_t* rx, int32_t* k,
                            int64_t* written) {
  return guard([&] {
    auto* ps = check_handle<sbr_paths_s>(p, kPaths, "paths");
    const int64_t n = ps->n_events;
    SBR_CHECK(capacity >= n, SBR_E_CAPACITY, "paths_events needs capacity %lld", (long long)n);
    set_device(ps->ctx);
    hipStream_t s = ps->ctx->stream;
    std::vector<uint32_t> r((size_t)n), qk((size_t)n);
    if (n > 0) {
      SBR_HIP(hipMemcpyAsync(r.data(), ps->ev_ray.p, n * 4, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipMemcpyAsync(qk.data(), ps->ev_qk.p, n * 4, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
    const sbr_trace_s* tr = ps->trace;
    const RayOrder ord{tr->R, (int32_t)tr->Nt, (int32_t)tr->emin};
    for (int64_t i = 0; i < n; ++i) {
      if (ray) ray[i] = (uint32_t)rid_of_pos(ord, (int64_t)r[i]);
      if (rx) rx[i] = (int32_t)(qk[i] >> 5);
      if (k) k[i] = (int32_t)(qk[i] & 31u);
    }
    if (written) *written = n;
  });
}

sbr_status sbr_paths_get(sbr_paths_t p, int64_t capacity, sbr_path_record* out, int64_t* written) {
  return guard([&] {
    auto* ps = check_handle<sbr_paths_s>(p, kPaths, "paths");
    const int64_t n = ps->n_paths;
    SBR_CHECK(capacity >= n, SBR_E_CAPACITY, "paths_get needs capacity %lld", (long long)n);
    SBR_CHECK(out != nullptr || n == 0, SBR_E_INVALID_ARG, "out is NULL");
    set_device(ps->ctx);
    hipStream_t s = ps->ctx->stream;
    const int K = ps->trace->K;
    std::vector<int32_t> key((size_t)n * (4 + K));
    std::vector<double> info((size_t)n * 2), pw((size_t)n);
    std::vector<float> ang((size_t)n * 4);
    if (n > 0) {
      SBR_HIP(hipMemcpyAsync(key.data(), ps->key.p, key.size() * 4, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipMemcpyAsync(info.data(), ps->info.p, info.size() * 8, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipMemcpyAsync(ang.data(), ps->ang.p, ang.size() * 4, hipMemcpyDeviceToHost, s));
      if (ps->have_power) SBR_HIP(hipMemcpyAsync(pw.data(), ps->power.p, pw.size() * 8, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
    for (int64_t i = 0; i < n; ++i) {
      sbr_path_record& r = out[i];
      std::memset(&r, 0, sizeof r);
      const int32_t* k = &key[i * (4 + K)];
      r.tx = k[0], r.rx = k[1], r.order = k[2], r.flags = k[3];
      for (int j = 0; j < SBR_MAX_BOUNCES; ++j) r.groups[j] = j < K ? k[4 + j] : -1;
      r.length_m = info[2 * i], r.delay_s = info[2 * i + 1];
      r.aod_az = ang[4 * i], r.aod_el = ang[4 * i + 1], r.aoa_az = ang[4 * i + 2], r.aoa_el = ang[4 * i + 3];
      r.power = ps->have_power ? (float)pw[i] : 0.0f;
    }
    if (written) *written = n;
  });
}

namespace {
struct FieldInputs {
  Buf f, adb, adeg;
  ChannelArgs a{};
};
void field_inputs(FieldInputs& F, const double* freq, int Nf, const float* atm_db, const float* atm_deg, int ptx,
                  int prx, uint32_t flags, hipStream_t s) {
  SBR_CHECK(Nf >= 1, SBR_E_INVALID_ARG, "Nf = %d", Nf);
  SBR_CHECK(ptx == SBR_POL_V || ptx == SBR_POL_H, SBR_E_INVALID_ARG, "pol_tx = %d", ptx);
  SBR_CHECK(prx == SBR_POL_V || prx == SBR_POL_H, SBR_E_INVALID_ARG, "pol_rx = %d", prx);
  const auto hf = to_host(freq, (size_t)Nf, flags, s);
  for (int i = 0; i < Nf; ++i)
    SBR_CHECK(std::isfinite(hf[i]) && hf[i] > 0, SBR_E_INVALID_ARG, "freq[%d] = %g", i, hf[i]);
  upload(F.f, freq, (size_t)Nf, flags, s);
  if (atm_db) upload(F.adb, atm_db, (size_t)Nf, flags, s);
  if (atm_deg) upload(F.adeg, atm_deg, (size_t)Nf, flags, s);
  F.a = ChannelArgs{F.f.as<double>(), atm_db ? F.adb.as<float>() : nullptr, atm_deg ? F.adeg.as<float>() : nullptr,
                    Nf, ptx, prx};
}
}  // namespace

sbr_status sbr_channel(sbr_context_t ctx, sbr_paths_t p, const double* freq, int32_t Nf, const float* atm_db,
                       const float* atm_deg, int32_t pol_tx, int32_t pol_rx, void* H_c64, double* H_c128,
                       uint32_t flags) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    auto* ps = check_handle<sbr_paths_s>(p, kPaths, "paths");
    set_device(c);
    hipStream_t s = c->stream;
    FieldInputs F;
    field_inputs(F, freq, Nf, atm_db, atm_deg, pol_tx, pol_rx, flags, s);
    const size_t nH = (size_t)Nf * ps->Nr * ps->trace->Nt;
    Buf t64, t128;
    float2* d64 = static_cast<float2*>(H_c64);
    double2* d128 = reinterpret_cast<double2*>(H_c128);
    const bool dev_out = flags & SBR_OUT_DEVICE;
    if (!dev_out) {
      if (H_c64) t64.alloc(nH * 8, s), d64 = t64.as<float2>();
      if (H_c128) t128.alloc(nH * 16, s), d128 = t128.as<double2>();
    }
    run_channel(ps, F.a, d64, d128, s);
    if (!dev_out) {
      if (H_c64) SBR_HIP(hipMemcpyAsync(H_c64, d64, nH * 8, hipMemcpyDeviceToHost, s));
      if (H_c128) SBR_HIP(hipMemcpyAsync(H_c128, d128, nH * 16, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
  });
}

sbr_status sbr_path_field(sbr_context_t ctx, sbr_paths_t p, const double* freq, int32_t Nf, const float* atm_db,
                          const float* atm_deg, int32_t pol_tx, int32_t pol_rx, double* a_c128, uint32_t flags) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    auto* ps = check_handle<sbr_paths_s>(p, kPaths, "paths");
    SBR_CHECK(a_c128 != nullptr || ps->n_paths == 0, SBR_E_INVALID_ARG, "output is NULL");
    set_device(c);
    hipStream_t s = c->stream;
    FieldInputs F;
    field_inputs(F, freq, Nf, atm_db, atm_deg, pol_tx, pol_rx, flags, s);
    const size_t n = (size_t)ps->n_paths * Nf;
    Buf tmp;
    double2* dst = reinterpret_cast<double2*>(a_c128);
    if (!(flags & SBR_OUT_DEVICE)) tmp.alloc(n * 16, s), dst = tmp.as<double2>();
    run_path_field(ps, F.a, dst, s);
    if (!(flags & SBR_OUT_DEVICE)) {
      if (n) SBR_HIP(hipMemcpyAsync(a_c128, dst, n * 16, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
  });
}

// ---------------------------------------------------------------- diffraction
sbr_status sbr_diffract(sbr_context_t ctx, sbr_scene_t scene, const double* tx_xyz, int32_t Nt, const double* rx_xyz,
                        int32_t Nr, uint32_t flags, sbr_diff_t* out) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    auto* sc = check_handle<sbr_scene_s>(scene, kScene, "scene");
    SBR_CHECK(out != nullptr, SBR_E_INVALID_ARG, "out is NULL");
    SBR_CHECK(Nt >= 1 && Nr >= 1 && (int64_t)Nt * Nr < (int64_t(1) << 31), SBR_E_INVALID_ARG, "Nt = %d, Nr = %d", Nt,
              Nr);
    SBR_CHECK(tx_xyz && rx_xyz, SBR_E_INVALID_ARG, "tx or rx is NULL");
    set_device(c);
    hipStream_t s = c->stream;
    const auto htx = to_host(tx_xyz, (size_t)Nt * 3, flags, s);
    const auto hrx = to_host(rx_xyz, (size_t)Nr * 3, flags, s);
    SBR_CHECK(finite_all(htx.data(), htx.size()) && finite_all(hrx.data(), hrx.size()), SBR_E_INVALID_ARG,
              "tx and rx coordinates must be finite");
    auto* d = new sbr_diff_s();
    d->ctx = c, d->scene = sc;
    retain(c), retain(sc);
    try {
      d->Nt = Nt, d->Nr = Nr;
      upload(d->tx, htx.data(), htx.size(), 0, s);
      upload(d->rx, hrx.data(), hrx.size(), 0, s);
      run_diffract(d, s);
    } catch (...) {
      release(d);
      throw;
    }
    *out = d;
  });
}

sbr_status sbr_diff_info(sbr_diff_t d, int64_t* wedges, int64_t* candidates, int64_t* geometric, int64_t* paths) {
  return guard([&] {
    auto* df = check_handle<sbr_diff_s>(d, kDiff, "diffraction");
    if (wedges) *wedges = df->scene->n_wedges;
    if (candidates) *candidates = df->n_candidates;
    if (geometric) *geometric = df->n_geometric;
    if (paths) *paths = df->n_paths;
  });
}

sbr_status sbr_diff_paths(sbr_diff_t d, int64_t capacity, int32_t* ids, double* rec, int64_t* written) {
  return guard([&] {
    auto* df = check_handle<sbr_diff_s>(d, kDiff, "diffraction");
    const int64_t n = std::min<int64_t>(capacity, df->n_paths);
    SBR_CHECK(n <= 0 || (ids && rec), SBR_E_INVALID_ARG, "output is NULL");
    set_device(df->ctx);
    hipStream_t s = df->ctx->stream;
    if (n > 0) {
      SBR_HIP(hipMemcpyAsync(ids, df->ids.p, (size_t)n * 12, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipMemcpyAsync(rec, df->rec.p, (size_t)n * 64, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
    if (written) *written = std::max<int64_t>(n, 0);
  });
}

sbr_status sbr_scene_wedges(sbr_context_t ctx, sbr_scene_t scene, int64_t capacity, double* geo, int32_t* groups,
                            int64_t* count) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    auto* sc = check_handle<sbr_scene_s>(scene, kScene, "scene");
    set_device(c);
    hipStream_t s = c->stream;
    scene_wedges(sc, s);
    if (count) *count = sc->n_wedges;
    const int64_t n = std::min<int64_t>(capacity, sc->n_wedges);
    if (n <= 0) return;
    SBR_CHECK(geo || groups, SBR_E_INVALID_ARG, "output is NULL");
    std::vector<WedgeDev> h((size_t)n);
    SBR_HIP(hipMemcpyAsync(h.data(), sc->wedges.p, (size_t)n * sizeof(WedgeDev), hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) {
      const WedgeDev& w = h[(size_t)i];
      if (geo) {
        double* g = geo + 8 * i;
        for (int k = 0; k < 3; ++k) g[k] = w.a[k], g[3 + k] = w.a[k] + w.len * w.e[k];
        g[6] = w.nw, g[7] = w.len;
      }
      if (groups) groups[2 * i] = w.g0, groups[2 * i + 1] = w.gn;
    }
  });
}

sbr_status sbr_diff_channel(sbr_context_t ctx, sbr_diff_t d, const double* freq, int32_t Nf, const float* atm_db,
                            const float* atm_deg, int32_t pol_tx, int32_t pol_rx, void* H_c64, double* H_c128,
                            uint32_t flags) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    auto* df = check_handle<sbr_diff_s>(d, kDiff, "diffraction");
    SBR_CHECK(H_c64 || H_c128, SBR_E_INVALID_ARG, "no output");
    set_device(c);
    hipStream_t s = c->stream;
    FieldInputs F;
    field_inputs(F, freq, Nf, atm_db, atm_deg, pol_tx, pol_rx, flags, s);
    const size_t nH = (size_t)Nf * df->Nr * df->Nt;
    Buf t64, t128;
    float2* d64 = static_cast<float2*>(H_c64);
    double2* d128 = reinterpret_cast<double2*>(H_c128);
    const bool dev_out = flags & SBR_OUT_DEVICE;
    if (!dev_out) {  // host H: add to a device copy of it
      if (H_c64) {
        t64.alloc(nH * 8, s), d64 = t64.as<float2>();
        SBR_HIP(hipMemcpyAsync(d64, H_c64, nH * 8, hipMemcpyHostToDevice, s));
      }
      if (H_c128) {
        t128.alloc(nH * 16, s), d128 = t128.as<double2>();
        SBR_HIP(hipMemcpyAsync(d128, H_c128, nH * 16, hipMemcpyHostToDevice, s));
      }
    }
    run_diff_channel(df, F.a.freq, Nf, F.a.atm_db, F.a.atm_deg, pol_tx, pol_rx, d64, d128, s);
    if (!dev_out) {
      if (H_c64) SBR_HIP(hipMemcpyAsync(H_c64, d64, nH * 8, hipMemcpyDeviceToHost, s));
      if (H_c128) SBR_HIP(hipMemcpyAsync(H_c128, d128, nH * 16, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
  });
}

sbr_status sbr_diff_field(sbr_context_t ctx, sbr_diff_t d, const double* freq, int32_t Nf, const float* atm_db,
                          const float* atm_deg, int32_t pol_tx, int32_t pol_rx, double* a_c128, uint32_t flags) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    auto* df = check_handle<sbr_diff_s>(d, kDiff, "diffraction");
    SBR_CHECK(a_c128 != nullptr || df->n_paths == 0, SBR_E_INVALID_ARG, "output is NULL");
    set_device(c);
    hipStream_t s = c->stream;
    FieldInputs F;
    field_inputs(F, freq, Nf, atm_db, atm_deg, pol_tx, pol_rx, flags, s);
    const size_t n = (size_t)df->n_paths * Nf;
    Buf tmp;
    double2* dst = reinterpret_cast<double2*>(a_c128);
    if (!(flags & SBR_OUT_DEVICE)) tmp.alloc(std::max<size_t>(n, 1) * 16, s), dst = tmp.as<double2>();
    run_diff_field(df, F.a.freq, Nf, F.a.atm_db, F.a.atm_deg, pol_tx, pol_rx, dst, s);
    if (!(flags & SBR_OUT_DEVICE)) {
      if (n) SBR_HIP(hipMemcpyAsync(a_c128, dst, n * 16, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
  });
}

sbr_status sbr_utd_transition(sbr_context_t ctx, const double* X, int64_t n, double* F_c128, uint32_t flags) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    SBR_CHECK(n >= 0 && (n == 0 || (X && F_c128)), SBR_E_INVALID_ARG, "transition arguments");
    if (n == 0) return;
    set_device(c);
    hipStream_t s = c->stream;
    Buf x, out;
    upload(x, X, (size_t)n, flags, s);
    double2* dst = reinterpret_cast<double2*>(F_c128);
    if (!(flags & SBR_OUT_DEVICE)) out.alloc((size_t)n * 16, s), dst = out.as<double2>();
    run_utd_transition(x.as<double>(), n, dst, s);
    if (!(flags & SBR_OUT_DEVICE)) {
      SBR_HIP(hipMemcpyAsync(F_c128, dst, (size_t)n * 16, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
  });
}

// ---------------------------------------------------------------- directive scattering
sbr_status sbr_scatter(sbr_context_t ctx, sbr_scene_t scene, const double* tx_xyz, int32_t Nt, const double* rx_xyz,
                       int32_t Nr, double tile_area, int32_t alpha, uint32_t flags, sbr_scat_t* out) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    auto* sc = check_handle<sbr_scene_s>(scene, kScene, "scene");
    SBR_CHECK(out != nullptr, SBR_E_INVALID_ARG, "out is NULL");
    SBR_CHECK(Nt >= 1 && Nr >= 1 && (int64_t)Nt * Nr < (int64_t(1) << 31), SBR_E_INVALID_ARG, "Nt = %d, Nr = %d", Nt,
              Nr);
    SBR_CHECK(tx_xyz && rx_xyz, SBR_E_INVALID_ARG, "tx or rx is NULL");
    SBR_CHECK(std::isfinite(tile_area) && tile_area > 0.0, SBR_E_INVALID_ARG, "tile_area = %g must be > 0",
              tile_area);
    SBR_CHECK(alpha >= 0 && alpha <= kMaxScatAlpha, SBR_E_INVALID_ARG, "alpha = %d outside [0, %d]", alpha,
              kMaxScatAlpha);
    set_device(c);
    hipStream_t s = c->stream;
    const auto htx = to_host(tx_xyz, (size_t)Nt * 3, flags, s);
    const auto hrx = to_host(rx_xyz, (size_t)Nr * 3, flags, s);
    SBR_CHECK(finite_all(htx.data(), htx.size()) && finite_all(hrx.data(), hrx.size()), SBR_E_INVALID_ARG,
              "tx and rx coordinates must be finite");
    auto* d = new sbr_scat_s();
    d->ctx = c, d->scene = sc;
    retain(c), retain(sc);
    try {
      d->Nt = Nt, d->Nr = Nr, d->alpha = alpha, d->tile_area = tile_area;
      upload(d->tx, htx.data(), htx.size(), 0, s);
      upload(d->rx, hrx.data(), hrx.size(), 0, s);
      run_scatter(d, s);
    } catch (...) {
      release(d);
      throw;
    }
    *out = d;
  });
}

sbr_status sbr_scat_info(sbr_scat_t d, int64_t* tiles, int64_t* candidates, int64_t* clear_legs, int64_t* paths) {
  return guard([&] {
    auto* df = check_handle<sbr_scat_s>(d, kScat, "scattering");
    if (tiles) *tiles = df->n_tiles;
    if (candidates) *candidates = df->n_candidates;
    if (clear_legs) *clear_legs = df->n_clear;
    if (paths) *paths = df->n_paths;
  });
}

sbr_status sbr_scat_paths(sbr_scat_t d, int64_t capacity, int32_t* ids, double* rec, int64_t* written) {
  return guard([&] {
    auto* df = check_handle<sbr_scat_s>(d, kScat, "scattering");
    const int64_t n = std::min<int64_t>(capacity, df->n_paths);
    SBR_CHECK(n <= 0 || (ids && rec), SBR_E_INVALID_ARG, "output is NULL");
    set_device(df->ctx);
    hipStream_t s = df->ctx->stream;
    if (n > 0) {
      SBR_HIP(hipMemcpyAsync(ids, df->ids.p, (size_t)n * 12, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipMemcpyAsync(rec, df->rec.p, (size_t)n * 16, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
    if (written) *written = std::max<int64_t>(n, 0);
  });
}

sbr_status sbr_scat_tiles(sbr_scat_t d, int64_t capacity, double* geo, int32_t* tri, int64_t* count) {
  return guard([&] {
    auto* df = check_handle<sbr_scat_s>(d, kScat, "scattering");
    if (count) *count = df->n_tiles;
    const int64_t n = std::min<int64_t>(capacity, df->n_tiles);
    if (n <= 0) return;
    SBR_CHECK(geo || tri, SBR_E_INVALID_ARG, "output is NULL");
    set_device(df->ctx);
    hipStream_t s = df->ctx->stream;
    std::vector<TileDev> h((size_t)n);
    SBR_HIP(hipMemcpyAsync(h.data(), df->tiles.p, (size_t)n * sizeof(TileDev), hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) {
      const TileDev& t = h[(size_t)i];
      if (geo) geo[4 * i] = t.c[0], geo[4 * i + 1] = t.c[1], geo[4 * i + 2] = t.c[2], geo[4 * i + 3] = t.ds;
      if (tri) tri[i] = t.tri;
    }
  });
}

sbr_status sbr_scat_channel(sbr_context_t ctx, sbr_scat_t d, const double* freq, int32_t Nf, const float* atm_db,
                            const float* atm_deg, int32_t pol_tx, int32_t pol_rx, void* H_c64, double* H_c128,
                            uint32_t flags) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    auto* df = check_handle<sbr_scat_s>(d, kScat, "scattering");
    SBR_CHECK(H_c64 || H_c128, SBR_E_INVALID_ARG, "no output");
    set_device(c);
    hipStream_t s = c->stream;
    FieldInputs F;
    field_inputs(F, freq, Nf, atm_db, atm_deg, pol_tx, pol_rx, flags, s);
    const size_t nH = (size_t)Nf * df->Nr * df->Nt;
    Buf t64, t128;
    float2* d64 = static_cast<float2*>(H_c64);
    double2* d128 = reinterpret_cast<double2*>(H_c128);
    const bool dev_out = flags & SBR_OUT_DEVICE;
    if (!dev_out) {  // host H: add to a device copy of it
      if (H_c64) {
        t64.alloc(nH * 8, s), d64 = t64.as<float2>();
        SBR_HIP(hipMemcpyAsync(d64, H_c64, nH * 8, hipMemcpyHostToDevice, s));
      }
      if (H_c128) {
        t128.alloc(nH * 16, s), d128 = t128.as<double2>();
        SBR_HIP(hipMemcpyAsync(d128, H_c128, nH * 16, hipMemcpyHostToDevice, s));
      }
    }
    run_scat_channel(df, F.a.freq, Nf, F.a.atm_db, F.a.atm_deg, pol_tx, pol_rx, d64, d128, s);
    if (!dev_out) {
      if (H_c64) SBR_HIP(hipMemcpyAsync(H_c64, d64, nH * 8, hipMemcpyDeviceToHost, s));
      if (H_c128) SBR_HIP(hipMemcpyAsync(H_c128, d128, nH * 16, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
  });
}

sbr_status sbr_scat_field(sbr_context_t ctx, sbr_scat_t d, const double* freq, int32_t Nf, const float* atm_db,
                          const float* atm_deg, int32_t pol_tx, int32_t pol_rx, double* a_c128, uint32_t flags) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    auto* df = check_handle<sbr_scat_s>(d, kScat, "scattering");
    SBR_CHECK(a_c128 != nullptr || df->n_paths == 0, SBR_E_INVALID_ARG, "output is NULL");
    set_device(c);
    hipStream_t s = c->stream;
    FieldInputs F;
    field_inputs(F, freq, Nf, atm_db, atm_deg, pol_tx, pol_rx, flags, s);
    const size_t n = (size_t)df->n_paths * Nf;
    Buf tmp;
    double2* dst = reinterpret_cast<double2*>(a_c128);
    if (!(flags & SBR_OUT_DEVICE)) tmp.alloc(std::max<size_t>(n, 1) * 16, s), dst = tmp.as<double2>();
    run_scat_field(df, F.a.freq, Nf, F.a.atm_db, F.a.atm_deg, pol_tx, pol_rx, dst, s);
    if (!(flags & SBR_OUT_DEVICE)) {
      if (n) SBR_HIP(hipMemcpyAsync(a_c128, dst, n * 16, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
  });
}

sbr_status sbr_scatter_lobe_norm(sbr_context_t ctx, int32_t alpha, const double* cos_i, int64_t n, double* out,
                                 uint32_t flags) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    SBR_CHECK(alpha >= 0 && alpha <= kMaxScatAlpha, SBR_E_INVALID_ARG, "alpha = %d outside [0, %d]", alpha,
              kMaxScatAlpha);
    SBR_CHECK(n >= 0 && (n == 0 || (cos_i && out)), SBR_E_INVALID_ARG, "lobe normalisation arguments");
    if (n == 0) return;
    set_device(c);
    hipStream_t s = c->stream;
    Buf x, o;
    upload(x, cos_i, (size_t)n, flags, s);
    double* dst = out;
    if (!(flags & SBR_OUT_DEVICE)) o.alloc((size_t)n * 8, s), dst = o.as<double>();
    run_lobe_norm(alpha, x.as<double>(), n, dst, s);
    if (!(flags & SBR_OUT_DEVICE)) {
      SBR_HIP(hipMemcpyAsync(out, dst, (size_t)n * 8, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
  });
}

sbr_status sbr_stats(sbr_paths_t p, float* pg_db, float* tau, float* angles, uint32_t flags) {
  return guard([&] {
    auto* ps = check_handle<sbr_paths_s>(p, kPaths, "paths");
    SBR_CHECK(ps->have_power, SBR_E_STATE, "sbr_stats needs a preceding sbr_channel");
    set_device(ps->ctx);
    hipStream_t s = ps->ctx->stream;
    const size_t nseg = (size_t)ps->Nr * ps->trace->Nt;
    if (flags & SBR_OUT_DEVICE) {
      run_stats(ps, pg_db, tau, angles, s);
      return;
    }
    Buf a, b, cbuf;
    if (pg_db) a.alloc(nseg * 4, s);
    if (tau) b.alloc(nseg * 4, s);
    if (angles) cbuf.alloc(nseg * 16, s);
    run_stats(ps, a.as<float>(), b.as<float>(), cbuf.as<float>(), s);
    if (pg_db) SBR_HIP(hipMemcpyAsync(pg_db, a.p, nseg * 4, hipMemcpyDeviceToHost, s));
    if (tau) SBR_HIP(hipMemcpyAsync(tau, b.p, nseg * 4, hipMemcpyDeviceToHost, s));
    if (angles) SBR_HIP(hipMemcpyAsync(angles, cbuf.p, nseg * 16, hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
  });
}

namespace {
// the set's Tx and Rx points must be the traced ones, bit for bit
void same_points(const Buf& tx, const Buf& rx, const std::vector<double>& htx, const Buf& prx, int Nt, int Nr,
                 const char* what, hipStream_t s) {
  std::vector<double> a((size_t)Nt * 3), b((size_t)Nr * 3), c((size_t)Nr * 3);
  SBR_HIP(hipMemcpyAsync(a.data(), tx.p, a.size() * 8, hipMemcpyDeviceToHost, s));
  SBR_HIP(hipMemcpyAsync(b.data(), rx.p, b.size() * 8, hipMemcpyDeviceToHost, s));
  SBR_HIP(hipMemcpyAsync(c.data(), prx.p, c.size() * 8, hipMemcpyDeviceToHost, s));
  SBR_HIP(hipStreamSynchronize(s));
  SBR_CHECK(std::memcmp(a.data(), htx.data(), a.size() * 8) == 0 && std::memcmp(b.data(), c.data(), b.size() * 8) == 0,
            SBR_E_INVALID_ARG, "the %s paths were found for other Tx or Rx points than the reflection paths", what);
}
}  // namespace

sbr_status sbr_stats_all(sbr_paths_t p, sbr_diff_t d, sbr_scat_t sc, float* pg_db, float* tau, float* angles,
                         uint32_t flags) {
  return guard([&] {
    auto* ps = check_handle<sbr_paths_s>(p, kPaths, "paths");
    SBR_CHECK(ps->have_power, SBR_E_STATE, "sbr_stats_all needs a preceding sbr_channel");
    sbr_diff_s* df = d ? check_handle<sbr_diff_s>(d, kDiff, "diffraction") : nullptr;
    sbr_scat_s* st = sc ? check_handle<sbr_scat_s>(sc, kScat, "scattering") : nullptr;
    const int Nt = ps->trace->Nt, Nr = ps->Nr;
    SBR_CHECK(!df || (df->Nt == Nt && df->Nr == Nr), SBR_E_INVALID_ARG, "diffraction paths of %d Tx x %d Rx, "
              "reflection paths of %d x %d", df ? df->Nt : 0, df ? df->Nr : 0, Nt, Nr);
    SBR_CHECK(!st || (st->Nt == Nt && st->Nr == Nr), SBR_E_INVALID_ARG, "scattering paths of %d Tx x %d Rx, "
              "reflection paths of %d x %d", st ? st->Nt : 0, st ? st->Nr : 0, Nt, Nr);
    SBR_CHECK(!df || df->have_power, SBR_E_STATE, "sbr_stats_all needs a preceding sbr_diff_channel");
    SBR_CHECK(!st || st->have_power, SBR_E_STATE, "sbr_stats_all needs a preceding sbr_scat_channel");
    set_device(ps->ctx);
    hipStream_t s = ps->ctx->stream;
    if (df) same_points(df->tx, df->rx, ps->trace->h_tx, ps->rx, Nt, Nr, "diffraction", s);
    if (st) same_points(st->tx, st->rx, ps->trace->h_tx, ps->rx, Nt, Nr, "scattering", s);
    StatSet sets[kMaxStatSets];
    int n = 0;
    sets[n++] = stat_set(ps);
    Buf dd, da, sd, sa;
    if (df) {
      const size_t m = (size_t)std::max<int64_t>(df->n_paths, 1);
      dd.alloc(m * 8, s), da.alloc(m * 16, s);
      run_diff_aux(df, dd.as<double>(), da.as<float>(), s);
      sets[n++] = StatSet{df->seg_start.as<int32_t>(), df->power.as<double>(), dd.as<double>(), 1, da.as<float>()};
    }
    if (st) {
      const size_t m = (size_t)std::max<int64_t>(st->n_paths, 1);
      sd.alloc(m * 8, s), sa.alloc(m * 16, s);
      run_scat_aux(st, sd.as<double>(), sa.as<float>(), s);
      sets[n++] = StatSet{st->seg_start.as<int32_t>(), st->power.as<double>(), sd.as<double>(), 1, sa.as<float>()};
    }
    const size_t nseg = (size_t)Nr * Nt;
    if (flags & SBR_OUT_DEVICE) {
      run_stats_sets(sets, n, (int64_t)nseg, pg_db, tau, angles, s);
      SBR_HIP(hipStreamSynchronize(s));  // the per-path records above are freed on return
      return;
    }
    Buf a, b, cbuf;
    if (pg_db) a.alloc(nseg * 4, s);
    if (tau) b.alloc(nseg * 4, s);
    if (angles) cbuf.alloc(nseg * 16, s);
    run_stats_sets(sets, n, (int64_t)nseg, a.as<float>(), b.as<float>(), cbuf.as<float>(), s);
    if (pg_db) SBR_HIP(hipMemcpyAsync(pg_db, a.p, nseg * 4, hipMemcpyDeviceToHost, s));
    if (tau) SBR_HIP(hipMemcpyAsync(tau, b.p, nseg * 4, hipMemcpyDeviceToHost, s));
    if (angles) SBR_HIP(hipMemcpyAsync(angles, cbuf.p, nseg * 16, hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
  });
}

sbr_status sbr_capacity(sbr_context_t ctx, const void* H_c64, int32_t Nf, int32_t Nr, int32_t Nt,
                        const double* snr_db, int32_t Nsnr, int32_t normalize, double* C, uint32_t flags) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    SBR_CHECK(Nf >= 1 && Nr >= 1 && Nt >= 1 && Nsnr >= 1, SBR_E_INVALID_ARG, "capacity sizes");
    SBR_CHECK(std::min(Nr, Nt) <= 128, SBR_E_UNSUPPORTED, "min(Nr, Nt) = %d > 128", std::min(Nr, Nt));
    SBR_CHECK(H_c64 && snr_db && C, SBR_E_INVALID_ARG, "NULL argument");
    set_device(c);
    hipStream_t s = c->stream;
    Buf h, sn, out;
    upload(h, static_cast<const float2*>(H_c64), (size_t)Nf * Nr * Nt, flags, s);
    upload(sn, snr_db, (size_t)Nsnr, flags, s);
    out.alloc((size_t)Nsnr * 8, s);
    run_capacity(h.as<float2>(), Nf, Nr, Nt, sn.as<double>(), Nsnr, normalize, out.as<double>(), s);
    SBR_HIP(hipMemcpyAsync(C, out.p, (size_t)Nsnr * 8,
                           (flags & SBR_OUT_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
  });
}

sbr_status sbr_port_power(sbr_context_t ctx, const void* H_c64, int32_t Nf, int32_t Nr, int32_t Nt, double* P,
                          uint32_t flags) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    SBR_CHECK(Nf >= 1 && Nr >= 1 && Nt >= 1, SBR_E_INVALID_ARG, "port power sizes");
    SBR_CHECK(H_c64 && P, SBR_E_INVALID_ARG, "NULL argument");
    set_device(c);
    hipStream_t s = c->stream;
    const size_t nq = (size_t)Nr * Nt;
    Buf h, out;
    const float2* Hd = static_cast<const float2*>(H_c64);
    if (!(flags & SBR_IN_DEVICE)) {
      upload(h, Hd, (size_t)Nf * nq, flags, s);
      Hd = h.as<float2>();
    }
    double* Pd = P;
    if (!(flags & SBR_OUT_DEVICE)) {
      out.alloc(nq * 8, s);
      Pd = out.as<double>();
    }
    run_port_power(Hd, Nf, Nr, Nt, Pd, s);
    if (!(flags & SBR_OUT_DEVICE)) {
      SBR_HIP(hipMemcpyAsync(P, Pd, nq * 8, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
  });
}

sbr_status sbr_capacity_noalloc(sbr_context_t ctx, const void* H_c64, int32_t Nf, int32_t Nr, int32_t Nt,
                                const double* snr_db, int32_t Nsnr, int32_t normalize, double* C) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    SBR_CHECK(Nf >= 1 && Nr >= 1 && Nt >= 1 && Nsnr >= 1, SBR_E_INVALID_ARG, "capacity sizes");
    SBR_CHECK(H_c64 && snr_db && C, SBR_E_INVALID_ARG, "NULL argument");
    SBR_CHECK(capacity_noalloc_fits(Nf, Nr, Nt, Nsnr), SBR_E_CAPACITY,
              "sbr_capacity_noalloc takes min(Nr, Nt) <= 128, Nsnr <= 64 and Nf * (Nsnr + 1) <= %lld "
              "(got Nf %d, Nr %d, Nt %d, Nsnr %d)",
              (long long)(kCapScratchBytes / 8 - 32), Nf, Nr, Nt, Nsnr);
    void* scratch = capacity_scratch(c->device);
    SBR_CHECK(scratch != nullptr, SBR_E_STATE, "capacity scratch of device %d not set up", c->device);
    set_device(c);
    run_capacity_noalloc(static_cast<const float2*>(H_c64), Nf, Nr, Nt, snr_db, Nsnr, normalize, C, scratch,
                         c->stream);
  });
}

sbr_status sbr_profile_enable(sbr_context_t ctx, int enable) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    set_device(c);
    c->prof.clear();
    c->prof.enabled = enable != 0;
  });
}

sbr_status sbr_profile_only(sbr_context_t ctx, const char* kernel) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    set_device(c);
    c->prof.clear();
    c->prof.only = kernel ? kernel : "";
  });
}

sbr_status sbr_profile_query(sbr_context_t ctx, const char* kernel, double* total_ms, int64_t* launches) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    SBR_CHECK(kernel != nullptr, SBR_E_INVALID_ARG, "kernel name is NULL");
    set_device(c);
    c->prof.resolve();
    double ms = 0.0;
    int64_t n = 0;
    for (auto& e : c->prof.acc)
      if (e.first == kernel) ms = e.second.first, n = e.second.second;
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
  });
}

sbr_status sbr_context_set_tuning(sbr_context_t ctx, const char* key, int32_t value) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    SBR_CHECK(key != nullptr, SBR_E_INVALID_ARG, "key is NULL");
    const std::string k(key);
    if (k == "trace_blocks_per_cu") {
      SBR_CHECK(value >= 1 && value <= 32, SBR_E_INVALID_ARG, "trace_blocks_per_cu = %d", value);
      c->tune.trace_blocks_per_cu = value;
    } else if (k == "trace_chunk") {
      SBR_CHECK(value >= 64 && value <= 4096 && value % 64 == 0, SBR_E_INVALID_ARG, "trace_chunk = %d", value);
      c->tune.trace_chunk = value;
    } else if (k == "trace_leaf_share") {
      SBR_CHECK(value >= 1 && value <= 64, SBR_E_INVALID_ARG, "trace_leaf_share = %d", value);
      c->tune.trace_leaf_share = value;
    } else if (k == "replay_block") {
      SBR_CHECK(value >= 64 && value <= 1024 && value % 64 == 0, SBR_E_INVALID_ARG, "replay_block = %d", value);
      c->tune.replay_block = value;
    } else if (k == "trace_graph") {
      SBR_CHECK(value == 0 || value == 1, SBR_E_INVALID_ARG, "trace_graph = %d", value);
      c->tune.trace_graph = value;
    } else if (k == "bvh_ploc_max") {
      SBR_CHECK(value >= 0 && value <= kBvhPlocMax, SBR_E_INVALID_ARG, "bvh_ploc_max = %d", value);
      c->tune.bvh_ploc_max = value;
    } else if (k == "trace_order") {
      SBR_CHECK(value == 0 || value == 1, SBR_E_INVALID_ARG, "trace_order = %d", value);
      c->tune.trace_order = value;
    } else if (k == "trace_packet") {
      SBR_CHECK(value == 0 || value == 1, SBR_E_INVALID_ARG, "trace_packet = %d", value);
      c->tune.trace_packet = value;
    } else if (k == "receive_event_capacity") {
      SBR_CHECK(value >= 0, SBR_E_INVALID_ARG, "receive_event_capacity = %d", value);
      c->tune.receive_event_capacity = value;
    } else {
      SBR_CHECK(false, SBR_E_INVALID_ARG, "unknown tuning key '%s'", key);
    }
  });
}

sbr_status sbr_context_get_tuning(sbr_context_t ctx, const char* key, int32_t* value) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    SBR_CHECK(key != nullptr && value != nullptr, SBR_E_INVALID_ARG, "NULL argument");
    const std::string k(key);
    if (k == "trace_blocks_per_cu") *value = c->tune.trace_blocks_per_cu;
    else if (k == "trace_chunk") *value = c->tune.trace_chunk;
    else if (k == "trace_leaf_share") *value = c->tune.trace_leaf_share;
    else if (k == "replay_block") *value = c->tune.replay_block;
    else if (k == "trace_graph") *value = c->tune.trace_graph;
    else if (k == "bvh_ploc_max") *value = c->tune.bvh_ploc_max;
    else if (k == "trace_order") *value = c->tune.trace_order;
    else if (k == "trace_packet") *value = c->tune.trace_packet;
    else if (k == "receive_event_capacity") *value = c->tune.receive_event_capacity;
    else SBR_CHECK(false, SBR_E_INVALID_ARG, "unknown tuning key '%s'", key);
  });
}

sbr_status sbr_context_count_work(sbr_context_t ctx, int enable) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    c->count_work = enable != 0;
  });
}

sbr_status sbr_trace_work(sbr_trace_t t, int64_t* node_visits, int64_t* tri_tests) {
  return guard([&] {
    auto* tr = check_handle<sbr_trace_s>(t, kTrace, "trace");
    set_device(tr->ctx);
    uint64_t w[2] = {0, 0};
    if (tr->counted) {
      SBR_HIP(hipMemcpyAsync(w, tr->work.p, 16, hipMemcpyDeviceToHost, tr->ctx->stream));
      SBR_HIP(hipStreamSynchronize(tr->ctx->stream));
    }
    if (node_visits) *node_visits = (int64_t)w[0];
    if (tri_tests) *tri_tests = (int64_t)w[1];
  });
}

sbr_status sbr_geodesic(sbr_context_t ctx, int32_t N, int64_t first, int64_t count, double* dirs, uint32_t flags) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    const int64_t R = 10LL * N * N + 2;
    SBR_CHECK(N >= 1 && N <= 46340 && first >= 0 && count >= 0 && first + count <= R, SBR_E_INVALID_ARG,
              "geodesic range");
    SBR_CHECK(dirs != nullptr || count == 0, SBR_E_INVALID_ARG, "dirs is NULL");
    set_device(c);
    hipStream_t s = c->stream;
    Buf tmp;
    double* dst = dirs;
    if (!(flags & SBR_OUT_DEVICE)) tmp.alloc((size_t)count * 24, s), dst = tmp.as<double>();
    launch_geodesic(N, first, count, dst, s);
    if (!(flags & SBR_OUT_DEVICE)) {
      if (count) SBR_HIP(hipMemcpyAsync(dirs, dst, (size_t)count * 24, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
  });
}

sbr_status sbr_geodesic_alpha(sbr_context_t ctx, int32_t N, double* mean, double* mn, double* mx) {
  return guard([&] {
    auto* c = check_handle<sbr_context_s>(ctx, kContext, "context");
    SBR_CHECK(N >= 1 && N <= 46340, SBR_E_INVALID_ARG, "N = %d", N);
    set_device(c);
    geodesic_edge_stats(N, mean, mn, mx, c->stream);
  });
}

}  // extern "C"
