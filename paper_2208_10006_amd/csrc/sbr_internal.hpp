// sbr_internal.hpp -- internal types of libsbr (not part of the C-ABI).
//
// Data layout in HBM (structure of arrays everywhere a kernel streams):
//   scene:  FP32 centred triangles in BVH leaf order (3 x float4 per
//           triangle: v0|tri id, v1|plane id, v2|group id), 64-byte BVH nodes
//           holding both child boxes, FP64 per-triangle planes (n, c) and
//           vertices for the exact FP64 steps, per-group plane/material and a
//           CSR of group members.
//   trace:  hit chain seq[k][ray] (int32, k-major so each bounce writes one
//           contiguous plane), ping-pong FP64 ray SoA between bounces.
//   paths:  per path a FP64 geometry record (stride 14 + 8K doubles) with the
//           frequency-independent polarisation chain, (rx, tx)-major order.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sbr.h"

namespace sbr {

// ----------------------------------------------------------------- constants
constexpr double kC0 = 299792458.0;        // m/s
constexpr double kEps0 = 8.8541878128e-12; // F/m
constexpr double kPi = 3.14159265358979323846;
constexpr int kWave = 64;

// path geometry record (FP64): header then 8 doubles per bounce
//   [0] length  [1] order k
//   [2..5]  c_init for V (2) and H (2): components of the Tx polarisation on (s_1, p_in_1)
//   [6..9]  w for V (2) and H (2): Rx polarisation on (s_k, p_out_k)
//   [10..13] line-of-sight e_rx . e_tx for VV, VH, HV, HH (k = 0)
//   bounce b: cos_i, eps_r, sigma, rough, G00, G01, G10, G11 (G maps (s_b,p_out_b)
//             amplitudes onto (s_{b+1}, p_in_{b+1}))
constexpr int kGeoHead = 14;
constexpr int kGeoPerBounce = 8;
inline int geo_stride(int K) { return kGeoHead + kGeoPerBounce * (K > 0 ? K : 1); }

// ----------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
struct Error {
  sbr_status st;
};

#define SBR_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      ::sbr::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
      throw ::sbr::Error{e_ == hipErrorOutOfMemory ? SBR_E_OUT_OF_MEMORY : SBR_E_DEVICE};  \
    }                                                                                      \
  } while (0)

#define SBR_CHECK(cond, status, ...)         \
  do {                                       \
    if (!(cond)) {                           \
      ::sbr::set_error(__VA_ARGS__);         \
      throw ::sbr::Error{status};            \
    }                                        \
  } while (0)

#define SBR_LAUNCH_CHECK() SBR_HIP(hipGetLastError())

// ----------------------------------------------------------------- handles
enum Kind : int { kContext = 0x5bc0, kScene, kTrace, kPaths, kDiff, kScat };

struct Handle {
  int kind;
  std::atomic<int> refs{1};
  explicit Handle(int k) : kind(k) {}
  virtual ~Handle() = default;
};
void retain(Handle* h);
void release(Handle* h);

// device buffer owned by a handle (stream-ordered allocation)
// Device buffer.  Blocks are stream-ordered allocations; a released block is
// kept in a per-stream cache and handed to the next allocation of a fitting
// size on the same stream without a HIP call (stream order makes the reuse
// safe), so the many short-lived temporaries of an API call cost no runtime
// calls once the sizes have been seen.  buf_cache_flush(stream) frees the
// cached blocks of a stream before it goes away.
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  size_t cap = 0;  // size of the block behind p
  hipStream_t stream = nullptr;
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  ~Buf() { reset(); }
  void alloc(size_t n, hipStream_t s);
  // a non-owning view of n bytes inside another Buf's block (reset() only forgets it)
  void view(void* base, size_t n) {
    reset();
    p = base, bytes = n;
  }
  void reset();
  template <class T> T* as() const { return static_cast<T*>(p); }
};
void buf_cache_flush(hipStream_t s);

// Live kernel timing: HIP events around launches, accumulated per kernel class.
struct Prof {
  bool enabled = false;
  std::string only;  // time only this kernel class (and no host phases); empty: everything
  struct Pending {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> spare;  // events returned by resolve(), reused by later launches
  std::vector<std::pair<std::string, std::pair<double, int64_t>>> acc;
  bool wants(const char* name) const { return enabled && (only.empty() || only == name); }
  void resolve();  // synchronises on the recorded events
  void clear();
  void destroy_events();
};
// the profiler of the context whose API call is running on this thread
extern thread_local Prof* g_prof;
struct TimedLaunch {
  hipEvent_t a = nullptr, b = nullptr;
  const char* name;
  hipStream_t s;
  TimedLaunch(const char* n, hipStream_t st);
  ~TimedLaunch();
};

// Wall time of a host-side phase, accumulated under "host:<name>" when profiling.
struct HostPhase {
  const char* name;
  double t0 = 0.0;
  explicit HostPhase(const char* n);
  ~HostPhase();
};
void prof_add(const char* name, double ms);

struct Tuning {
  int trace_blocks_per_cu = 4; // resident 256-thread blocks per CU of the persistent grid
  int trace_chunk = 64;        // rays per wave per queue pull (64 or 128)
  int trace_leaf_share = 40;   // 64ths of a wave's tracing lanes holding leaves before they are tested together
  int replay_block = 256;
  int trace_graph = 0;         // 1: replay the bounce loop as a cached hipGraph
  int bvh_ploc_max = 65536;    // scenes up to this many triangles are clustered with PLOC
  int trace_order = 1;         // 1: element-minor ray positions for traces of several elements (RayOrder)
  int trace_packet = 0;        // 1: the wave traverses the tree as one (single-scene traces)
  int receive_event_capacity = 0;  // initial capture-event capacity of a receive; 0: max(2^20, rays / 8)
};

// An instantiated bounce-loop graph: init kernels + one kernel node per bounce,
// built once per shape and replayed with updated kernel arguments.
struct TraceGraph {
  int K = -1, depth_bucket = 0, count = 0, packet = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipGraphNode_t> nodes;  // fill counters, bounce 0..K
  ~TraceGraph();
};

}  // namespace sbr

namespace sbr {
// Pinned host memory for uploads and for copies of device inputs, with an
// event that marks the end of a scene build's input copies.
struct HostStage {
  void* p = nullptr;
  size_t bytes = 0;
  hipEvent_t ev = nullptr;
  void reserve(size_t need);  // grows only; never while copies from it are in flight
  HostStage() = default;
  HostStage(const HostStage&) = delete;
  HostStage& operator=(const HostStage&) = delete;
  ~HostStage();
};
// a stream and staging area of the batched scene build (one per worker thread)
struct SceneWorker {
  hipStream_t stream = nullptr;
  HostStage stage;
};
}  // namespace sbr

struct sbr_context_s : sbr::Handle {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int num_cus = 256;
  sbr::Tuning tune;
  sbr::Prof prof;
  bool count_work = false;
  sbr::HostStage stage;  // pinned host staging for this context's stream
  std::vector<sbr::SceneWorker*> workers;  // batched scene builds (created on first use)
  std::vector<sbr::TraceGraph*> graphs;  // cached bounce-loop graphs
  // grow-only device scratch reused by successive calls on this context's
  // stream (the two ray buffers of a trace); large per-call allocations from
  // the stream-ordered pool can stall while the pool grows
  sbr::Buf scratch[2];
  void* scratch_get(int slot, size_t bytes, hipStream_t s);
  sbr_context_s() : Handle(sbr::kContext) {}
  ~sbr_context_s() override;
};

struct sbr_scene_s : sbr::Handle {
  sbr_context_s* ctx = nullptr;
  int64_t T = 0;
  int n_groups = 0, n_planes = 0, bvh_depth = 0;
  // triangles in the BVH (leaves 0 .. n_bvh-1 of tri32) and oversized ones
  // kept out of it (tri32 entries n_bvh .. T-1, tested by every ray directly)
  int64_t n_bvh = 0;
  int n_big = 0;
  double center[3] = {0, 0, 0};
  double diag = 0.0;
  float root_host[6] = {0, 0, 0, 0, 0, 0};
  std::vector<int32_t> h_group, h_plane;
  sbr::Buf nodes;    // float4[4] per internal node (T-1, at least 1 when T >= 1)
  sbr::Buf root_box; // float[8]
  sbr::Buf tri32;    // float4[3] per triangle in leaf order
  sbr::Buf tri64;    // double[9] per triangle, original order, absolute coordinates
  sbr::Buf tplane;   // double4 per triangle: n, c (absolute coordinates)
  sbr::Buf tgroup;   // int per triangle
  sbr::Buf tplaneid; // int per triangle
  sbr::Buf gplane;   // double4 per group (plane of its lowest triangle)
  sbr::Buf gmat;     // float4 per group: eps_r, sigma, rough, 0
  sbr::Buf gstart;   // int[G+1]
  sbr::Buf gtri;     // int[T]
  sbr::Buf tables;   // one block holding tplane .. gtri (those are views into it)
  // wedge edges for diffraction (sbr::WedgeDev), built on first use
  std::mutex wedge_mu;
  bool have_wedges = false;
  int64_t n_wedges = 0;
  sbr::Buf wedges;
  // hand every buffer to stream s (built on a worker stream that has finished:
  // releases then follow the order of the stream that uses the scene)
  void rehome(hipStream_t s) {
    for (sbr::Buf* b : {&nodes, &root_box, &tri32, &tri64, &tplane, &tgroup, &tplaneid, &gplane, &gmat, &gstart,
                        &gtri, &tables, &wedges})
      if (b->p) b->stream = s;
  }
  sbr_scene_s() : Handle(sbr::kScene) {}
  ~sbr_scene_s() override;
};

struct sbr_trace_s : sbr::Handle {
  sbr_context_s* ctx = nullptr;
  sbr_scene_s* scene = nullptr;
  int Nt = 0, N = 0, K = 0;
  int emin = 0;  // ray positions in element-minor order (RayOrder)
  int64_t R = 0, NR = 0;
  std::vector<double> h_tx;
  sbr::Buf tx;      // double[Nt][3]
  sbr::Buf seq;     // int32[(K+1)][NR]
  sbr::Buf counters; // uint32: trace_counter_words(K), one block per bounce
  sbr::Buf work;     // uint64[2]: node visits, triangle tests (when counted)
  bool counted = false;
  int64_t segments = -1;  // host copy once read
  bool batched = false;   // traced by sbr_trace_batch (segments counted from the chains)
  double latency_ms = -1.0;
  sbr_trace_s() : Handle(sbr::kTrace) {}
  ~sbr_trace_s() override;
};

struct sbr_paths_s : sbr::Handle {
  sbr_context_s* ctx = nullptr;
  sbr_trace_s* trace = nullptr;
  int Nr = 0;
  double alpha = 0, coeff = 1;
  int64_t n_events = 0, n_keys = 0, n_paths = 0;
  sbr::Buf rx;        // double[Nr][3]
  sbr::Buf key;       // int32[n][4 + K]: tx, rx, k, flags, g_1..g_K
  sbr::Buf geo;       // double[n][stride]
  sbr::Buf info;      // double[n][2]: length, delay
  sbr::Buf ang;       // float[n][4]: aod az/el, aoa az/el (deg)
  sbr::Buf power;     // double[n] band-mean |a|^2
  sbr::Buf seg_start; // int32[Nr*Nt + 1]
  sbr::Buf ev_ray;    // uint32[n_events] capture events (kept for diagnostics)
  sbr::Buf ev_qk;     // uint32[n_events]: rx << 5 | k
  bool have_power = false;
  sbr_paths_s() : Handle(sbr::kPaths) {}
  ~sbr_paths_s() override;
};

// First-order edge-diffraction paths of one (scene, Tx set, Rx set).
struct sbr_diff_s : sbr::Handle {
  sbr_context_s* ctx = nullptr;
  sbr_scene_s* scene = nullptr;
  int Nt = 0, Nr = 0;
  int64_t n_candidates = 0, n_geometric = 0, n_paths = 0;
  sbr::Buf tx, rx;      // double[N][3]
  sbr::Buf ids;         // int32[n][3]: tx, rx, wedge (ordered by rx, tx, wedge)
  sbr::Buf rec;         // double[n][8]: Q xyz, s', s, beta0, phi', phi
  sbr::Buf seg_start;   // int32[Nr*Nt + 1]
  sbr::Buf power;       // double[n]: band power of each path in the last sbr_diff_channel
  bool have_power = false;
  sbr_diff_s() : Handle(sbr::kDiff) {}
  ~sbr_diff_s() override;
};

// First-order directive scattering paths of one (scene, tile area, exponent,
// Tx set, Rx set).
struct sbr_scat_s : sbr::Handle {
  sbr_context_s* ctx = nullptr;
  sbr_scene_s* scene = nullptr;
  int Nt = 0, Nr = 0, alpha = 0;
  double tile_area = 0.0;
  int64_t n_tiles = 0, n_candidates = 0, n_clear = 0, n_paths = 0;
  sbr::Buf tx, rx;      // double[N][3]
  sbr::Buf tiles;       // sbr::TileDev[n_tiles]
  sbr::Buf lobe;        // double[alpha / 2 + 1][alpha + 1]: lobe normalisation table
  sbr::Buf ids;         // int32[n][3]: tx, rx, tile (ordered by rx, tx, tile)
  sbr::Buf rec;         // double[n][2]: r_i, r_s
  sbr::Buf seg_start;   // int32[Nr*Nt + 1]
  sbr::Buf power;       // double[n]: band power of each path in the last sbr_scat_channel
  bool have_power = false;
  sbr_scat_s() : Handle(sbr::kScat) {}
  ~sbr_scat_s() override;
};

namespace sbr {

// ----------------------------------------------------------------- launchers
// sort.hip
size_t radix_sort_temp_bytes(int64_t n);
// Stable LSD sort of (key, val) by key bits [bit_lo, bit_hi); results in
// keys_out/vals_out (inputs are clobbered).  temp from radix_sort_temp_bytes.
void radix_sort_pairs(uint64_t* keys_in, uint32_t* vals_in, uint64_t* keys_out, uint32_t* vals_out, int64_t n,
                      int bit_lo, int bit_hi, void* temp, hipStream_t s);
size_t scan_temp_bytes(int64_t n);
// exclusive scan of uint32 (in place allowed); total written to *total_dev if non-null
void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev, void* temp,
                        hipStream_t s);
void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void iota_u32(uint32_t* p, int64_t n, hipStream_t s);
void gather_u64(const uint64_t* src, const uint32_t* idx, uint64_t* dst, int64_t n, hipStream_t s);

// face_groups.hip: plane (n, c) of every triangle in; group and plane id of
// every triangle, and their counts, out.  eps, sig, rough: materials [T].
struct Plane {
  double n[3], c;
};
void face_groups(const std::vector<Plane>& pl, const float* eps, const float* sig, const float* rough, double diag,
                 std::vector<int32_t>& group, std::vector<int32_t>& plane, int& ngroups, int& nplanes);

// bvh.hip: BVH over n primitives given their FP32 boxes (lo, hi) -> nodes,
// leaf permutation (sorted position -> primitive), root box.  PLOC clustering
// up to kBvhPlocMax primitives unless `linear` is set, Karras LBVH otherwise.
// Returns the depth.
constexpr int64_t kBvhPlocMax = 65536;
struct BvhOut {
  float4* nodes;     // [max(n-1,1)][4]
  uint32_t* order;   // [n] primitive of each leaf
  float* root_box;   // [8]
  float* root_host;  // optional host copy of the root box (6 floats), filled before return
  // optional: asynchronous build.  The depth is written to this device word
  // and build_bvh returns 0 without synchronising (root_host is not filled).
  uint32_t* depth_dev = nullptr;
  // optional: scene bounds (lo xyz, hi xyz) in device memory, used for the
  // Morton codes instead of scene_lo / scene_hi (which may then be null)
  const float* bounds_dev = nullptr;
};
// Linear trees of up to kLbvhSmall primitives are built by one workgroup.
// A root-to-leaf path has at most 41 internal nodes: along it the common
// prefix of the (30-bit code, 11-bit index) keys grows at every node.
constexpr int kLbvhSmall = 2048;
int build_bvh(const float* box_lo, const float* box_hi, int64_t n, const float scene_lo[3],
              const float scene_hi[3], BvhOut out, hipStream_t s, bool linear = false);

// geodesic.hip
void upload_geodesic_tables(int device);
void launch_geodesic(int N, int64_t first, int64_t count, double* dirs, hipStream_t s);
void geodesic_edge_stats(int N, double* mean, double* mn, double* mx, hipStream_t s);

// trace.hip
struct TraceLaunch {
  sbr_context_s* ctx;
  const sbr_scene_s* scene;
  const double* tx;
  int Nt, N, K;
  int emin;
  int64_t R, NR;
  int32_t* seq;
  uint32_t* counters;  // trace_counter_words(K): one kCtrWords block per bounce
  unsigned long long* work;  // node visits, triangle tests, or null (no counting)
  int grid, block, chunk, leaf_share;
  int packet;  // wave-uniform traversal (ignored when counting work)
};
void launch_trace(const TraceLaunch& L, void* ray_a, void* ray_b, hipStream_t s);
// one persistent launch per bounce over the rays of all traces (their seq,
// tx, N, K and scenes set); per-trace first/last wall-clock stamps
void launch_trace_batch(const std::vector<sbr_trace_s*>& trs, int grid, int chunk, int leaf_share, void* ray_a,
                        void* ray_b, uint32_t* counters, unsigned long long* t_first, unsigned long long* t_last,
                        hipStream_t s);
size_t trace_ray_bytes(int64_t NR);
// FP32 triangles in leaf order: kTriVecs float4 per triangle, its three
// vertices in each of the three cyclic axis orders (x y z | y z x | z x y),
// the .w lanes holding the original id, plane id and group id (vertex 0, 1, 2)
constexpr int kTriVecs = 9;

// Trace counters: per bounce a block of kCtrWords words holding, for each of
// the 8 ray regions x, the queue position (kCtrQueue + 32 x), the number of
// survivors written (kCtrOut + 32 x) and an "empty" flag (kCtrDone + 32 x).
constexpr int kCtrQueue = 0, kCtrOut = 256, kCtrDone = 512, kCtrWords = 1024;
int64_t trace_counter_words(int K);

// receive.hip
void run_receive(sbr_paths_s* ps, const double* hrx, hipStream_t s);  // hrx: host copy of the Rx points (null for sets of up to kLbvhSmall, prepared on the device)

// channel.hip
struct ChannelArgs {
  const double* freq;
  const float* atm_db;
  const float* atm_deg;
  int Nf, pol_tx, pol_rx;
};
void run_channel(sbr_paths_s* ps, const ChannelArgs& a, float2* H64, double2* H128, hipStream_t s);
void run_path_field(sbr_paths_s* ps, const ChannelArgs& a, double2* out, hipStream_t s);
void run_stats(sbr_paths_s* ps, float* pg_db, float* tau, float* angles, hipStream_t s);
void run_capacity(const float2* H, int Nf, int Nr, int Nt, const double* snr_db, int Nsnr, int normalize,
                  double* C_out, hipStream_t s);
// P[q][p] = band mean of |H_f[q][p]|^2 (FP64), H [Nf][Nr][Nt]
void run_port_power(const float2* H, int Nf, int Nr, int Nt, double* P, hipStream_t s);
// allocation-free capacity: a fixed device array of kCapScratchBytes per GPU
constexpr size_t kCapScratchBytes = size_t(8) << 20;
constexpr int kMaxDevices = 64;
void capacity_scratch_setup(int device);  // once per device, with it current (context creation)
void* capacity_scratch(int device);       // its address on `device`, or null before setup
bool capacity_noalloc_fits(int Nf, int Nr, int Nt, int Nsnr);
void run_capacity_noalloc(const float2* H, int Nf, int Nr, int Nt, const double* snr_db_host, int Nsnr,
                          int normalize, double* C_out, void* scratch, hipStream_t s);

// per-link statistics over several path sets (channel.hip): a set is a CSR
// per (rx, tx) pair, each path's band power, its delay at delay[n * dstride]
// and its angles [n][4] (departure azimuth, elevation, arrival azimuth,
// elevation, degrees)
struct StatSet {
  const int32_t* seg_start;
  const double* power;
  const double* delay;
  int dstride;
  const float* ang;
};
constexpr int kMaxStatSets = 3;
StatSet stat_set(sbr_paths_s* ps);
void run_stats_sets(const StatSet* sets, int nsets, int64_t nseg, float* pg_db, float* tau, float* angles,
                    hipStream_t s);
// power[n] = (1 / Nf) sum over tiles of part[n * ntiles + tile], tiles in order
void run_power_final(const double* part, int64_t n, int ntiles, int Nf, double* power, hipStream_t s);

// diffract.hip (first-order edge diffraction)
// one wedge edge: start point a, unit edge direction e, unit vector t0 in face 0
// perpendicular to the edge, unit normal n0 of face 0 on the exterior side,
// edge length, exterior angle / pi, face groups of face 0 and face n
struct WedgeDev {
  double a[3], e[3], t0[3], n0[3];
  double len, nw;
  int32_t g0, gn;
};
void scene_wedges(sbr_scene_s* sc, hipStream_t s);  // builds sc->wedges once (thread-safe)
void run_diffract(sbr_diff_s* d, hipStream_t s);
// H[f][q][p] += the diffracted field of every path (H64 and/or H128 may be null)
void run_diff_channel(sbr_diff_s* d, const double* freq, int Nf, const float* atm_db, const float* atm_deg, int ptx,
                      int prx, float2* H64, double2* H128, hipStream_t s);
void run_diff_field(sbr_diff_s* d, const double* freq, int Nf, const float* atm_db, const float* atm_deg, int ptx,
                    int prx, double2* out, hipStream_t s);
void run_utd_transition(const double* X, int64_t n, double2* out, hipStream_t s);
// [global ray id][K+1][2] barycentric (u, v) of every hit, NaN after the chain ends (receive.hip)
void run_hits_uv(sbr_trace_s* tr, float* uv, hipStream_t s);
// per path: delay (s) and angles [n][4] (degrees) for the per-link statistics
void run_diff_aux(sbr_diff_s* d, double* delay, float* ang, hipStream_t s);

// scatter.hip (first-order directive scattering)
// one surface tile: centroid, unit normal of its triangle, area, triangle and
// face group
struct TileDev {
  double c[3], n[3];
  double ds;
  int32_t tri, group;
};
void run_scatter(sbr_scat_s* d, hipStream_t s);
// H[f][q][p] += the scattered field of every path (H64 and/or H128 may be null)
void run_scat_channel(sbr_scat_s* d, const double* freq, int Nf, const float* atm_db, const float* atm_deg, int ptx,
                      int prx, float2* H64, double2* H128, hipStream_t s);
void run_scat_field(sbr_scat_s* d, const double* freq, int Nf, const float* atm_db, const float* atm_deg, int ptx,
                    int prx, double2* out, hipStream_t s);
void run_lobe_norm(int alpha, const double* cos_i, int64_t n, double* out, hipStream_t s);
void run_scat_aux(sbr_scat_s* d, double* delay, float* ang, hipStream_t s);
constexpr int kMaxScatAlpha = 32;

// nn.hip (surrogate)
// mask (bf16, may be null): the product is zeroed where mask[i*ldm + j] <= 0;
// bsum (may be null): bsum[j] = sum_k B(k,j) from the same FP32 accumulation
void nn_gemm(int M, int N, int K, const void* A, int64_t a_si, int64_t a_sk, const void* B, int64_t b_sk,
             int64_t b_sj, const float* bias, void* C, int64_t ldc, uint32_t flags, hipStream_t s,
             const void* mask = nullptr, int64_t ldm = 0, float* bsum = nullptr);
void nn_im2col(const void* x, int n, int H, int W, int C, void* col, hipStream_t s);
// y == null: dx (FP32) = adjoint of im2col; else dz_bf (bf16) = that sum where y > 0, else 0
void nn_col2im(const float* dcol, int n, int H, int W, int C, float* dx, hipStream_t s, const void* y = nullptr,
               void* dz_bf = nullptr);
void nn_fourier(const float* x, int64_t n, int D, int L, const void* emb, int E, const int32_t* scene,
                const float* extra, int X, int F, void* out, hipStream_t s);
void nn_mlp_fused(int64_t n, const void* shared, const void* emb, const int32_t* scene, const void* wt,
                  const float* bias, int depth, const void* out_w, const float* out_b, int T, float* out,
                  hipStream_t s);
void nn_transpose(const void* src, int rows, int cols, void* dst, hipStream_t s);
void nn_link_features(const float* raw, int64_t n, const int32_t* scene, const void* hmap, int H, float half,
                      int samples, float* x, float* extra, hipStream_t s);
void nn_relu_bwd(const float* g, const void* y, int64_t n, float* gout, void* gbf, hipStream_t s);
void nn_relu_bwd_colsum(const float* g, const void* y, int64_t M, int N, float* gout, void* gbf, float* colsum,
                        hipStream_t s);
void nn_cast(const float* a, int64_t n, void* b, hipStream_t s);
void nn_mse(const float* pred, int64_t ldp, const float* target, const float* weight, int64_t n, int T, float scale,
            float* dpred, int64_t ldd, double* loss, hipStream_t s);
void nn_colsum(const float* g, int64_t M, int N, int64_t ld, float* out, int accumulate, hipStream_t s);
void nn_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
             float wd, int step, void* wbf, hipStream_t s);
void nn_gather_rows(const void* src, int64_t row_bytes, const int64_t* idx, int64_t n, void* dst, hipStream_t s);
void nn_onehot(const int32_t* idx, int64_t n, int width, void* out, hipStream_t s);
void nn_ensemble(const float* out, int E, int64_t member_stride, int64_t n, int64_t ld, int t, float threshold,
                 float* mean, float* spread, uint8_t* mask, hipStream_t s);

}  // namespace sbr
