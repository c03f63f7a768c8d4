// C ABI of libstglbm (declared in include/stglbm.h).
//
// Host-side duties only: validate arguments, carve the caller's workspace,
// choose the launch shape, sequence the kernels on the caller's stream, move
// data for the test/ops helpers and report device flags.  Every step of the
// method runs in the kernels of lattice_kernels.hip and inlet_kernels.hip.
#include "stglbm.h"
#include <rocprofiler-sdk-roctx/roctx.h>

#include "stglbm_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace stglbm;

// Static device scratch of stglbm_step_noalloc: the inlet planes of the steps
// it is about to take.  Every GPU the library runs on holds one copy of it
// until the process ends; every call on a GPU shares that GPU's copy.
static constexpr uint64_t kScratchBytes = 16ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kVersion = 10000;        // 1.0.0
constexpr uint64_t kAlign = 256;
constexpr uint32_t kCkptMagic = 0x5354474cu;   // "STGL"
constexpr uint32_t kCkptVersion = 4;   // 2: store order [NZ][Q][NY][NX]; 3: velocity set and operator;
                                       // 4: 16-bit stores keep FP64 totals and FP32 window sums

thread_local std::string g_lib_error;

// Device address of `scratch` per device (looked up once per device).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// roctx range over a host entry point (shown by rocprofv3 --marker-trace).
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

struct Layout {
  uint64_t g[2] = {0, 0}, stats = 0, win = 0, sponge = 0, flag = 0, ubc = 0, rans = 0, rows = 0, modes = 0,
           sqrtq = 0, arow = 0, bz = 0, sig = 0, ptab = 0, scalars = 0, total = 0;
  int vec = 1, nxt = 0, wx = 1, wz = 1, nxg = 0, slots = 0, lw = 0, zstep = 1, nblocks = 0;
  bool short_chunks_when_idle = true;   // steps without statistics: their own shape
  int wx_idle = 1, nxg_idle = 1, lw_idle = 1;
  int remap_env = -1, lockstep = 1;   // tuning overrides read once per handle (-1: no override)
  int zsched = 0;                     // statistics launches: unequal z chunks, slot s on rows zbeg[s] .. zbeg[s + 1] - 1
  int zbeg[kMaxZChunks + 1] = {};
  int tail_planes = 1;                // statistics launches may make the next inlet plane in trailing blocks
  int f32_ilp = 0;                    // FP32 D3Q19 statistics launches: the max-ilp build of the kernel
};

uint64_t align_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int store_bytes(int store) { return store == STGLBM_F32 ? 4 : 2; }

// Populations of the descriptor's velocity set (0 selects D3Q19).
int set_size(const stglbm_lattice_desc* d) { return d->velocity_set == 0 ? 19 : d->velocity_set; }

// The step kernel addresses one z slice of the store ([Q][NY][NX] values)
// through a raw buffer resource of at most 4 GiB - 1.
bool slice_fits(const stglbm_lattice_desc* d) {
  return static_cast<uint64_t>(set_size(d)) * d->nx * d->ny * store_bytes(d->store) <= 0xffffffffull;
}

const char* check_desc(const stglbm_lattice_desc* d) {
  if (!d) return "null descriptor";
  if (d->nx < 2 || d->ny < 2 || d->nz < 1) return "lattice must have nx >= 2, ny >= 2, nz >= 1";
  if (static_cast<long long>(d->nx) * d->ny * d->nz > 0x7fffffffLL) return "lattice has 2^31 cells or more";
  if (d->store < 0 || d->store > 2) return "unknown store type";
  if (d->velocity_set != 0 && d->velocity_set != 15 && d->velocity_set != 19 && d->velocity_set != 27)
    return "velocity_set must be 15, 19 or 27 (0 = 19)";
  if (d->collision != 0 && d->collision != 1) return "collision must be 0 (regularized) or 1 (BGK)";
  if (!slice_fits(d)) return "lattice too large: one z slice (Q NY NX values) must stay below 4 GiB";
  if (!(d->nu_lb > 0.0) || !std::isfinite(d->nu_lb)) return "nu_lb must be positive";
  if (!(d->cs_smag >= 0.0)) return "cs_smag must be >= 0";
  if (!d->periodic_x) {
    if (d->max_modes < 1 || d->max_rans < 2) return "an inlet channel needs max_modes >= 1 and max_rans >= 2";
    if (!(d->rho_out > 0.0)) return "rho_out must be positive";
    if (d->sponge_cells < 0 || d->sponge_cells >= d->nx - 1) return "sponge_cells out of range";
  }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(d->force[a])) return "force must be finite";
  return nullptr;
}

// Rows of the row-phasor table: NY rounded up to a multiple of 8 (the most
// rows a plane block takes), so a block's last row group stays inside.
int ptab_rows(int ny) { return (ny + 7) / 8 * 8; }

// Statistics launches of 16-bit stores in whole-row blocks of 8 waves: MI355X
// holds 3 such blocks per compute unit (the kernel stays at <= 80 VGPRs), 768
// on its 256 CUs.  Their z chunks are cut unequal, longest first, so that the
// blocks dispatched last are short and the launch's tail is short too.
//
// When 768 is a whole number spr >= 3 of slots (blocks per slot = base, the
// x groups times NY), the z rows go into 2 spr chunks that fill exactly two
// rounds of resident blocks: spr long chunks first, spr - 2 slightly shorter
// ones, then 2 short ones (about half a mean chunk), which the positions
// that free up last take.  Fewer slots than the uniform rule's (12 against 16
// on 512x128x256) also mean fewer window-sum bytes per launch.  Measured on
// 512x128x256 FP16 (ms per step, one box): 24 x 6, 22 x 4, 12 x 2 rows 0.2575
// against 0.2633 for 16 chunks of 16; neighbours of that schedule
// 0.2578-0.2586; 11 chunks (a round of 5 slots) 0.272.
//
// Otherwise, where the uniform rule's S chunks make at least two rounds of
// blocks, the first half of them are long and the rest 0.6 of that length.
// Measured on 1024x256x512 FP16 (base 512, 4 chunks): 160, 160, 96, 96 rows
// 2.067 ms per step against 2.098 for 4 x 128 (120, 120, 104, 104, 64: 2.064;
// 96 x 4, 64 x 2: 2.067; 200, 200, 112: 2.088; 176, 176, 160: 2.108).
//
// Returns false (uniform chunks) where neither applies.
bool make_chunk_schedule(const stglbm_lattice_desc* d, Layout& L, int base) {
  constexpr int kResident = 3 * 256;
  if (d->store == STGLBM_F32 || L.wz != 1 || L.wx * L.wz != 8 || base <= 0) return false;
  const int nz = d->nz;
  int chunk[kMaxZChunks];
  int n = 0;
  if (kResident % base == 0 && kResident / base >= 3) {
    const int spr = kResident / base;
    n = 2 * spr;
    if (n > kMaxZChunks || nz < 4 * (n - 1)) return false;
    const int small = (nz + (n - 1)) / (2 * (n - 1));               // about half of nz / (n - 1)
    const int rest = nz - 2 * small;
    const int c1 = (rest + (n - 2) - 1) / (n - 2);                  // first round, rounded up
    const int r2 = rest - spr * c1;                                 // rows left for the spr - 2 middle chunks
    if (r2 < (spr - 2) * small) return false;
    for (int i = 0; i < spr; ++i) chunk[i] = c1;
    for (int i = 0; i < spr - 2; ++i) chunk[spr + i] = r2 / (spr - 2) + (i < r2 % (spr - 2) ? 1 : 0);
    chunk[n - 2] = chunk[n - 1] = small;
  } else {
    n = L.slots;
    if (n < 2 || n > kMaxZChunks || static_cast<long long>(base) * n < 2 * kResident) return false;
    const int h = (n + 1) / 2, t = n - h;
    const int a = static_cast<int>(std::lround(nz / (h + 0.6 * t)));
    const int r = nz - a * h;                                       // rows of the t short chunks
    if (a < 2 || r < t || r > a * t) return false;
    for (int i = 0; i < h; ++i) chunk[i] = a;
    for (int i = 0; i < t; ++i) chunk[h + i] = r / t + (i < r % t ? 1 : 0);
  }
  L.zbeg[0] = 0;
  for (int i = 0; i < n; ++i) L.zbeg[i + 1] = L.zbeg[i] + chunk[i];
  if (L.zbeg[n] != nz) return false;
  int longest = 0;
  for (int i = 0; i < n; ++i) longest = std::max(longest, chunk[i]);
  L.zsched = 1;
  L.slots = n;
  L.lw = longest;
  return true;
}

Layout make_layout(const stglbm_lattice_desc* d) {
  Layout L;
  const uint64_t cells = static_cast<uint64_t>(d->nx) * d->ny * d->nz;
  // Each lane owns vec consecutive x cells (1, 2 or 4).  Wider lanes make
  // 8-byte accesses but need more registers, and on MI355X one cell per lane
  // streams fastest at the channel sizes measured, so 1 is the default.
  int vec = 1;
  // Block shape: wx waves along x (consecutive tiles of 64 vec cells of one
  // row) times wz waves along z, each wave stepping lw cells in z.  Default:
  // whole rows of up to 512 vec cells per block, one wave deep (two for the
  // FP32 statistics launches of D3Q15 / D3Q19), lw as below.
  int wx = 0;
  int wz = 1;
  int lw = 0;
  int interleave = 0;
  if (const char* env = std::getenv("STGLBM_SHAPE")) {   // "wx,wz,lw[,vec[,interleave]]" tuning override
    int a = 0, b = 0, c = 0, v = 0, il = 1;
    const int n = std::sscanf(env, "%d,%d,%d,%d,%d", &a, &b, &c, &v, &il);
    if (n >= 3 && a >= 1 && b >= 1 && a * b <= kMaxWavesPerBlock && c >= 0) {
      wx = a; wz = b; lw = c;
      L.short_chunks_when_idle = false;
      if (n >= 4 && (v == 1 || v == 2 || v == 4) && d->nx % v == 0) vec = v;
      if (n >= 5) interleave = il ? 1 : 0;
    }
  }
  if (set_size(d) != 19 || d->collision != 0) vec = 1;   // the variants are built for one cell per lane
  if (const char* env = std::getenv("STGLBM_REMAP")) L.remap_env = std::atoi(env) ? 1 : 0;
  if (const char* env = std::getenv("STGLBM_LOCKSTEP")) L.lockstep = std::atoi(env) ? 1 : 0;
  if (const char* env = std::getenv("STGLBM_TAIL_STG")) L.tail_planes = std::atoi(env) ? 1 : 0;
  if (const char* env = std::getenv("STGLBM_F32_ILP")) L.f32_ilp = std::atoi(env) ? 1 : 0;
  L.vec = vec;
  L.nxt = (d->nx + 64 * vec - 1) / (64 * vec);
  const int wx_row = L.nxt < 8 ? L.nxt : 8;   // whole rows of up to 8 tiles
  L.wx_idle = wx == 0 ? wx_row : wx;
  if (wx == 0) wx = wx_row;   // whole rows of up to 8 tiles for both launch kinds
  L.wx = wx;
  L.wz = wz;
  L.nxg = (L.nxt + wx - 1) / wx;
  const int base = L.nxg * d->ny;
  const bool lw_default = lw == 0;
  if (lw == 0) {
    // Each block takes one contiguous z chunk; the blocks sharing an (x, y)
    // bin are its FP64 slots.  FP32 on D3Q15 / D3Q19 with one cell per lane:
    // two z waves per block (whole rows, 16 waves: one block fills a CU's
    // wave slots, so all its waves run in step and finish together), 2 slots,
    // more where the grid would hold fewer than 4096 waves.  Other FP32 sets:
    // one z wave, 4 slots.  16-bit stores: one z wave and as many slots as
    // make 16384 waves, then cut unequal (make_chunk_schedule).  Measured on
    // MI355X, 512x128x256: FP32 0.455 ms (two z waves and 4 slots 0.457; one
    // z wave: 4 slots 0.476, 8: 0.482, 16: 0.494; half rows with four z waves
    // 0.477-0.479); with one z wave the two 8-wave blocks sharing a CU ran at
    // different speeds, and the first to finish left the CU half empty for
    // the last 10-25 % of the launch.  Uniform chunks, FP16 with FP64 slots:
    // 16 slots 0.273 ms (8 slots 0.274, 4 slots 0.278, two z waves 0.298,
    // half rows 0.299); 1024x256x512 FP16 (4 slots) 2.098 ms (8 slots 2.103,
    // 16 slots 2.143, 2 slots 2.171): both best at 16384 waves.
    const bool f32 = d->store == STGLBM_F32;
    if (L.short_chunks_when_idle && step_max_waves(store_bytes(d->store), set_size(d), vec, true) == kMaxWavesWide) wz = 2;
    L.wz = wz;
    const int zmax = (d->nz + wz - 1) / wz;
    const int waves = base * wx * wz;
    const int min_waves = f32 ? 4096 : 16384, min_slots = wz == 2 ? 2 : (f32 ? 4 : 1);
    int slots = (min_waves + waves - 1) / waves;
    if (slots < min_slots) slots = min_slots;
    if (slots > zmax) slots = zmax;
    lw = (d->nz + wz * slots - 1) / (wz * slots);
  }
  L.lw = lw;
  L.slots = (d->nz + wz * lw - 1) / (wz * lw);
  const char* zenv = std::getenv("STGLBM_ZCHUNKS");   // "r0,r1,...": z rows per chunk, or "uniform" (tuning override)
  if (!zenv) {
    if (lw_default) make_chunk_schedule(d, L, base);
  } else if (std::strcmp(zenv, "uniform") != 0) {
    int beg[kMaxZChunks + 1] = {0}, n = 0, maxc = 0;
    bool ok = true;
    for (const char* c = zenv; *c && ok;) {
      char* end = nullptr;
      const long r = std::strtol(c, &end, 10);
      if (end == c || r <= 0 || r % wz != 0 || n >= kMaxZChunks) { ok = false; break; }
      beg[n + 1] = beg[n] + static_cast<int>(r);
      maxc = std::max(maxc, static_cast<int>(r));
      ++n;
      c = *end == ',' ? end + 1 : end;
    }
    if (ok && n > 0 && beg[n] == d->nz) {
      L.zsched = 1;
      std::copy(beg, beg + n + 1, L.zbeg);
      L.slots = n;
      L.lw = maxc / wz;
      interleave = 0;
    }
  }
  // Without statistics the z chunk only sets the block size.  Measured on
  // MI355X, the fastest blocks stream about 2 KB of each population row for
  // FP32 (one z row of 512 cells: 0.477 ms; two: 0.481) and about 4 KB for
  // 16-bit stores (512x128x256: 4 rows 0.268 ms, 2 rows 0.271, 1 row 0.303;
  // 1024x256x512 in half-row blocks: 4 rows 2.10 ms, 2 rows 2.17, 1 row 2.39).
  const int block_row_bytes = std::min(d->nx, L.wx_idle * 64 * vec) * store_bytes(d->store);
  const int target = d->store == STGLBM_F32 ? 2048 : 4096;
  L.lw_idle = std::max(1, (target + block_row_bytes - 1) / block_row_bytes);
  L.nxg_idle = (L.nxt + L.wx_idle - 1) / L.wx_idle;
  L.zstep = interleave ? L.slots * wz : wz;
  L.nblocks = base * L.slots;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const uint64_t gbytes = static_cast<uint64_t>(set_size(d)) * cells * store_bytes(d->store);
  L.g[0] = take(gbytes);
  L.g[1] = take(gbytes);
  // Statistics: FP64 totals and FP32 sums per slot over the current window
  // (kStatsWindow sampled steps).  The two pieces are adjacent, before the
  // sponge table.
  const uint64_t bins9 = 9ull * d->nx * d->ny;
  L.stats = take(bins9 * sizeof(double));
  L.win = take(static_cast<uint64_t>(L.slots) * bins9 * sizeof(float));
  L.sponge = take(static_cast<uint64_t>(d->nx) * sizeof(float));
  L.flag = take(2 * sizeof(int));
  if (!d->periodic_x) {
    L.ubc = take(static_cast<uint64_t>(kStgBatch) * d->ny * d->nz * 3 * sizeof(float));
    L.rans = take(static_cast<uint64_t>(d->max_rans) * 12 * sizeof(double));
    L.rows = take(static_cast<uint64_t>(d->ny) * kRowFields * sizeof(double));
    L.modes = take(static_cast<uint64_t>(d->max_modes) * kModeFields * sizeof(double));
    L.sqrtq = take(static_cast<uint64_t>(d->ny) * d->max_modes * sizeof(double));
    L.arow = take(static_cast<uint64_t>(d->ny) * d->max_modes * 2 * sizeof(double));
    L.bz = take(static_cast<uint64_t>(d->max_modes) * d->nz * sizeof(float2));
    L.sig = take(static_cast<uint64_t>(d->max_modes) * sizeof(float4));
    L.ptab = take(static_cast<uint64_t>(kStgBatch) * d->max_modes * ptab_rows(d->ny) * sizeof(float2));
    L.scalars = take(kScalars * sizeof(double));
  }
  L.total = off;
  return L;
}

uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

struct CkptHeader {
  uint32_t magic, version;
  int32_t nx, ny, nz, store, periodic_x, slots;
  uint64_t inlet_hash;
  int64_t t, n_samples;
  int32_t sampling, n_modes;
  uint64_t g_bytes, stats_bytes;
  int32_t q, collision;
};

}  // namespace

struct stglbm_ctx {
  stglbm_lattice_desc d{};
  Layout L;
  hipStream_t stream = nullptr;
  int device = -1;                 // device holding the workspace
  char* ws = nullptr;
  int cur = 0;
  int64_t t = 0;
  int64_t n_samples = 0;
  bool sampling = false;
  bool inlet_ready = false;
  int n_modes = 0;
  uint64_t inlet_hash = 0;
  double c_x = 0, c_t = 0, U_b = 0, L_e = 0;
  std::string err;
  bool prof = false;
  int prof_every = 1;          // time one step-kernel launch in prof_every
  int64_t prof_count = 0;
  std::vector<hipEvent_t> ev_step, ev_stg;   // start/stop pairs
  int n_probes = 0;                           // velocity probes (caller's device buffer)
  int probe_xyz[kMaxProbes][3] = {};
  float* probe_out = nullptr;
  int64_t probe_capacity = 0, probe_rows = 0;
  size_t n_step = 0, n_stg = 0, n_planes = 0, n_tail_planes = 0;
  // Inlet planes of the steps ring_t0 .. ring_t0 + ring_n - 1 held in the
  // ring of kStgBatch planes (step t in slot (t - ring_base) mod kStgBatch),
  // made ahead of use by a plane-kernel launch or by the trailing blocks of a
  // stream-collide launch (ring_n = 0: none valid).
  int64_t ring_t0 = 0, ring_base = 0;
  int ring_n = 0;
  // Row phasors of the steps ptab_t0 .. ptab_t0 + ptab_n - 1, in the table of
  // kStgBatch slots (step t in slot (t - ptab_base) mod kStgBatch), which the
  // plane kernel and the trailing plane blocks read (ptab_n = 0: none valid).
  int64_t ptab_t0 = 0, ptab_base = 0;
  int ptab_n = 0;

  template <class T> T* at(uint64_t off) { return reinterpret_cast<T*>(ws + off); }
  void* gbuf(int k) { return ws + L.g[k]; }
  uint64_t cells() const { return static_cast<uint64_t>(d.nx) * d.ny * d.nz; }
  int q() const { return set_size(&d); }
  uint64_t gbytes() const { return static_cast<uint64_t>(q()) * cells() * store_bytes(d.store); }
  uint64_t plane_floats() const { return static_cast<uint64_t>(d.ny) * d.nz * 3; }
};

namespace {

int fail(stglbm_t h, int code, const std::string& msg) {
  if (h) h->err = msg; else g_lib_error = msg;
  return code;
}

int hip_fail(stglbm_t h, hipError_t e, const char* what) {
  return fail(h, STGLBM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_CHECK(h, expr, what)                  \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(h, e_, what); \
  } while (0)

// Wait for the stream and turn device flags into an error.
int sync_and_check(stglbm_t h) {
  HIP_CHECK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  int flag = 0;
  HIP_CHECK(h, hipMemcpy(&flag, h->at<int>(h->L.flag), sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy flag");
  if (flag & kFlagDensity) return fail(h, STGLBM_E_UNSTABLE, "density deviation out of (-0.5, 0.5) or NaN in the lattice");
  if (flag & kFlagInletMach) return fail(h, STGLBM_E_UNSTABLE, "inlet velocity |u_x| >= 0.3 c_s");
  return STGLBM_OK;
}

// Timing events of the profiler.  They are only read after the stream has
// been synchronized, so they skip the system-scope fence (a cache write-back
// and invalidate at every record, about 8 us per step of two launches).
hipEvent_t pooled_event(std::vector<hipEvent_t>& pool, size_t idx) {
  while (pool.size() <= idx) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    pool.push_back(e);
  }
  return pool[idx];
}

StepParams step_params(stglbm_t h) {
  StepParams p{};
  const stglbm_lattice_desc& d = h->d;
  p.gin = h->gbuf(h->cur);
  p.gout = h->gbuf(1 - h->cur);
  p.plane2d = static_cast<long long>(d.nx) * d.ny;
  p.nx = d.nx; p.ny = d.ny; p.nz = d.nz;
  p.q = h->q();
  p.collision = d.collision;
  p.vec = h->L.vec;
  p.nxt = h->L.nxt; p.wx = h->L.wx; p.wz = h->L.wz; p.nxg = h->L.nxg;
  p.slots = h->L.slots; p.lw = h->L.lw; p.zstep = h->L.zstep; p.nblocks = h->L.nblocks;
  if (h->sampling && h->L.zsched) {
    p.zsched = 1;
    std::copy(h->L.zbeg, h->L.zbeg + h->L.slots + 1, p.zbeg);
  }
  if (!h->sampling && (h->L.short_chunks_when_idle || h->L.zsched)) {
    // The block shape and z chunk serve the statistics reduction (they set the
    // number of FP64 slots).  Without statistics, whole-row blocks with short
    // chunks stream fastest: the resident blocks then cover a narrow
    // contiguous band of z slices.
    p.wx = h->L.wx_idle;
    p.wz = 1;
    p.nxg = h->L.nxg_idle;
    p.lw = h->L.lw_idle;
    p.slots = (d.nz + p.lw - 1) / p.lw;
    p.zstep = 1;
    p.nblocks = p.nxg * d.ny * p.slots;
  }
  // One block per row (nxg = 1): the hardware's turn-by-turn XCD order is
  // kept (a contiguous range per XCD measured 3 % slower on 512x128x256).
  p.remap = (p.nxg > 1 && p.nblocks % (8 * p.nxg) == 0) ? 1 : 0;
  if (h->L.remap_env >= 0) p.remap = h->L.remap_env && p.nxg > 1 && p.nblocks % (8 * p.nxg) == 0;
  // Statistics launches keep their waves in step (512x128x256: FP32 with two
  // z waves 0.514 -> 0.458 ms, FP16 0.289 -> 0.273 ms).
  p.lockstep = h->L.lockstep;
  p.periodic_x = d.periodic_x;
  p.has_force = (d.force[0] != 0.0 || d.force[1] != 0.0 || d.force[2] != 0.0) ? 1 : 0;
  const double tau0 = 0.5 + 3.0 * d.nu_lb;
  p.tau0 = static_cast<float>(tau0);
  p.tau0_sq = static_cast<float>(tau0 * tau0);
  p.s0 = static_cast<float>(3.0 * d.nu_lb);
  p.c18 = static_cast<float>(18.0 * std::sqrt(2.0) * d.cs_smag * d.cs_smag);
  p.fx = static_cast<float>(d.force[0]);
  p.fy = static_cast<float>(d.force[1]);
  p.fz = static_cast<float>(d.force[2]);
  p.rho_out_m1 = static_cast<float>(d.rho_out - 1.0);
  p.inv_rho_out = static_cast<float>(1.0 / d.rho_out);
  p.mach_limit = static_cast<float>(0.3 / std::sqrt(3.0));
  p.sponge = h->at<float>(h->L.sponge);
  p.ubc = nullptr;   // set per step from the plane ring
  p.stats = h->at<double>(h->L.stats);
  p.win = h->at<float>(h->L.win);
  p.win_first = 0;
  p.flag = h->at<int>(h->L.flag);
  p.f32_ilp = h->L.f32_ilp;
  return p;
}

// Ring slot of the inlet plane of step t.
float* ring_slot(stglbm_t h, int64_t t) {
  const int64_t k = ((t - h->ring_base) % kStgBatch + kStgBatch) % kStgBatch;
  return h->at<float>(h->L.ubc) + static_cast<uint64_t>(k) * h->plane_floats();
}

// Plane parameters of the n consecutive steps t_first .. t_first + n - 1,
// written one after the other to out.
StgParams stg_params(stglbm_t h, int64_t t_first, int n, float* out) {
  StgParams s{};
  s.modes = h->at<double>(h->L.modes);
  s.arow = h->at<double2>(h->L.arow);
  s.bz = h->at<float2>(h->L.bz);
  s.sig = h->at<float4>(h->L.sig);
  s.rows = h->at<double>(h->L.rows);
  s.out = out;
  s.ptab = h->at<float2>(h->L.ptab);
  s.ptab_rows = ptab_rows(h->d.ny);
  s.ny = h->d.ny; s.nz = h->d.nz; s.n_modes = h->n_modes;
  s.n_planes = n;
  for (int b = 0; b < n; ++b)
    s.pslot[b] = static_cast<int>(((t_first + b - h->ptab_base) % kStgBatch + kStgBatch) % kStgBatch);
  s.c_x = h->c_x;
  s.conv = h->c_t / h->c_x;
  const double kTwoPi = 6.283185307179586476925;
  for (int b = 0; b < n; ++b)
    s.tphase[b] = kTwoPi * (0.0 - h->U_b * (static_cast<double>(t_first + b) * h->c_t)) / h->L_e;
  return s;
}

// Row phasors of the steps t_first .. t_first + n - 1 (n <= kStgBatch) in the
// table; if any is missing, those of the kStgBatch steps from t_first are made
// first (one small launch, on the handle's stream before their readers).
int ensure_row_phases(stglbm_t h, int64_t t_first, int n) {
  if (h->ptab_n > 0 && t_first >= h->ptab_t0 && t_first + n <= h->ptab_t0 + h->ptab_n) return STGLBM_OK;
  h->ptab_n = 0;
  h->ptab_t0 = h->ptab_base = t_first;
  HIP_CHECK(h, launch_stg_time_phase(stg_params(h, t_first, kStgBatch, nullptr), h->stream), "STG row-phase launch");
  h->ptab_n = kStgBatch;
  return STGLBM_OK;
}

// STG planes of the n consecutive steps t_first .. t_first + n - 1, written
// one after the other to out (n <= kStgBatch), in one launch.
int launch_planes(stglbm_t h, int64_t t_first, int n, float* out, bool timed_ok = true) {
  if (int rc = ensure_row_phases(h, t_first, n)) return rc;
  const StgParams s = stg_params(h, t_first, n, out);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = timed_ok && h->prof;
  if (timed) {
    e0 = pooled_event(h->ev_stg, 2 * h->n_stg);
    e1 = pooled_event(h->ev_stg, 2 * h->n_stg + 1);
    if (e0 && e1) HIP_CHECK(h, hipEventRecord(e0, h->stream), "hipEventRecord");
  }
  HIP_CHECK(h, launch_stg(s, h->stream), "STG plane kernel launch");
  if (timed && e0 && e1) {
    HIP_CHECK(h, hipEventRecord(e1, h->stream), "hipEventRecord");
    ++h->n_stg;
    h->n_planes += static_cast<size_t>(n);
  }
  return STGLBM_OK;
}

// Inlet plane of step t (device pointer into the ring), generating the next
// kStgBatch planes first if t is not held.
int ring_plane(stglbm_t h, int64_t t, const float** plane) {
  if (h->ring_n == 0 || t < h->ring_t0 || t >= h->ring_t0 + h->ring_n) {
    h->ring_n = 0;
    if (int rc = launch_planes(h, t, kStgBatch, h->at<float>(h->L.ubc))) return rc;
    h->ring_t0 = h->ring_base = t;
    h->ring_n = kStgBatch;
  }
  *plane = ring_slot(h, t);
  return STGLBM_OK;
}

// One time step: the fused stream-collide launch reading the inlet plane
// `plane` (null for periodic x), the buffer swap and the probes.  With
// `timed`, the profiler's events may bracket the launch (they are created on
// first use, so the allocation-free entry point passes false).  With
// `ring_ahead`, a statistics launch without a body force also makes the plane
// of step t + 2 in its trailing blocks when the ring holds planes up to t + 1
// (ring steps need blocks of at least kStgWaves waves).
int step_once(stglbm_t h, const float* plane, bool timed_ok, bool ring_ahead = false) {
  StepParams p = step_params(h);
  p.ubc = plane;
  const int64_t t2 = h->t + 2;
  const bool tail = ring_ahead && h->L.tail_planes && plane && h->sampling && !p.has_force &&
                    h->d.store != STGLBM_F32 && p.wx * p.wz >= kStgWaves &&
                    h->ring_n > 0 && h->ring_t0 + h->ring_n == t2 && h->ring_t0 <= h->t + 1;
  if (tail) {
    p.stg_zb = (h->d.nz + 63) / 64;
    p.stg_blocks = p.stg_zb * ((h->d.ny + kStgTailRows - 1) / kStgTailRows);
    if (int rc = ensure_row_phases(h, t2, 1)) return rc;
    p.stg = stg_params(h, t2, 1, ring_slot(h, t2));
  }
  const bool window = h->sampling;
  if (window) p.win_first = h->n_samples % kStatsWindow == 0 ? 1 : 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = timed_ok && h->prof && (h->prof_count++ % h->prof_every == 0);
  if (timed) {
    e0 = pooled_event(h->ev_step, 2 * h->n_step);
    e1 = pooled_event(h->ev_step, 2 * h->n_step + 1);
    if (e0 && e1) HIP_CHECK(h, hipEventRecord(e0, h->stream), "hipEventRecord");
  }
  HIP_CHECK(h, launch_step(p, h->d.store, h->sampling, h->stream), "step kernel launch");
  if (timed && e0 && e1) {
    HIP_CHECK(h, hipEventRecord(e1, h->stream), "hipEventRecord");
    ++h->n_step;
  }
  if (tail) {
    // plane t + 2 replaces the one kStgBatch steps earlier in its slot
    const int64_t end = t2 + 1;
    h->ring_t0 = std::max(h->ring_t0, end - kStgBatch);
    h->ring_n = static_cast<int>(end - h->ring_t0);
    if (h->prof) ++h->n_tail_planes;   // counted like the other profile figures, while profiling
  }
  h->cur = 1 - h->cur;
  ++h->t;
  if (h->sampling) ++h->n_samples;
  if (window && h->n_samples % kStatsWindow == 0) {
    // fold the window's FP32 slot sums into the FP64 totals, slots in order
    HIP_CHECK(h, launch_stats_sum(nullptr, 0, h->at<float>(h->L.win), h->L.slots, 9ll * h->d.nx * h->d.ny,
                                  h->at<double>(h->L.stats), true, h->stream),
              "statistics fold");
  }
  if (h->n_probes > 0 && h->probe_rows < h->probe_capacity) {
    ProbeParams q{};
    q.g = h->gbuf(h->cur);
    q.plane2d = static_cast<long long>(h->d.nx) * h->d.ny;
    q.q = h->q();
    q.nx = h->d.nx;
    q.n = h->n_probes;
    q.fx = h->d.force[0];
    q.fy = h->d.force[1];
    q.fz = h->d.force[2];
    std::memcpy(q.xyz, h->probe_xyz, sizeof(q.xyz));
    q.out = h->probe_out + 3 * h->n_probes * h->probe_rows;
    HIP_CHECK(h, launch_probes(q, h->d.store, h->stream), "probe kernel launch");
    ++h->probe_rows;
  }
  return STGLBM_OK;
}

// Device address of `scratch` on the handle's device.  The array's name is a
// host-side stand-in; its device address is looked up once per device, with
// that device current, and kept.
int device_scratch(stglbm_t h, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (h->device < 0 || h->device >= kMaxDevices) return fail(h, STGLBM_E_HIP, "step_noalloc: unknown device of the workspace");
  if (!g_scratch_ptr[h->device]) {
    int prev = 0;
    HIP_CHECK(h, hipGetDevice(&prev), "hipGetDevice");
    if (prev != h->device) HIP_CHECK(h, hipSetDevice(h->device), "hipSetDevice");
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != h->device) (void)hipSetDevice(prev);
    if (e != hipSuccess || !ptr) return hip_fail(h, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[h->device] = ptr;
  }
  *out = g_scratch_ptr[h->device];
  return STGLBM_OK;
}

}  // namespace

extern "C" {

int stglbm_version(void) { return kVersion; }

const char* stglbm_status_string(int s) {
  switch (s) {
    case STGLBM_OK: return "ok";
    case STGLBM_E_INVAL: return "invalid argument";
    case STGLBM_E_NOMEM: return "workspace too small";
    case STGLBM_E_HIP: return "HIP error";
    case STGLBM_E_STATE: return "call out of order";
    case STGLBM_E_UNSTABLE: return "instability detected";
    case STGLBM_E_REALIZABILITY: return "Reynolds stress not realizable";
    default: return "unknown status";
  }
}

int stglbm_derive_units(double delta, int32_t ny, double u_b_lb, double U_b, double nu_phys,
                        double* c_x, double* c_t, double* nu_lb) {
  if (!(delta > 0) || ny < 1 || !(u_b_lb > 0) || !(U_b > 0) || !(nu_phys > 0) || !c_x || !c_t || !nu_lb)
    return fail(nullptr, STGLBM_E_INVAL, "derive_units: arguments must be positive");
  *c_x = 2.0 * delta / ny;
  *c_t = u_b_lb * (*c_x) / U_b;
  *nu_lb = nu_phys * (*c_t) / ((*c_x) * (*c_x));
  return STGLBM_OK;
}

int stglbm_acceleration_to_lattice(double c_x, double c_t, const double* a_phys, double* force_lb) {
  if (!a_phys || !force_lb) return fail(nullptr, STGLBM_E_INVAL, "acceleration_to_lattice: null array");
  if (!(c_x > 0.0) || !(c_t > 0.0) || !std::isfinite(c_x) || !std::isfinite(c_t))
    return fail(nullptr, STGLBM_E_INVAL, "acceleration_to_lattice: c_x and c_t must be positive");
  for (int a = 0; a < 3; ++a) force_lb[a] = a_phys[a] * c_t * c_t / c_x;
  return STGLBM_OK;
}

int stglbm_footprint(const stglbm_lattice_desc* desc, uint64_t* bytes) {
  if (const char* m = check_desc(desc)) return fail(nullptr, STGLBM_E_INVAL, m);
  if (!bytes) return fail(nullptr, STGLBM_E_INVAL, "null output");
  *bytes = make_layout(desc).total;
  return STGLBM_OK;
}

int stglbm_init_lattice(const stglbm_lattice_desc* desc, void* d_workspace, uint64_t ws_bytes,
                        void* hip_stream, stglbm_t* out) {
  if (!out) return fail(nullptr, STGLBM_E_INVAL, "null handle output");
  *out = nullptr;
  if (const char* m = check_desc(desc)) return fail(nullptr, STGLBM_E_INVAL, m);
  if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) % kAlign))
    return fail(nullptr, STGLBM_E_INVAL, "workspace must be non-null and 256-byte aligned");
  Layout L = make_layout(desc);
  if (ws_bytes < L.total) return fail(nullptr, STGLBM_E_NOMEM, "workspace smaller than stglbm_footprint()");
  stglbm_t h = new (std::nothrow) stglbm_ctx();
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "host allocation failed");
  h->d = *desc;
  h->L = L;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->ws = static_cast<char*>(d_workspace);
  {
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, d_workspace) == hipSuccess && attr.device >= 0) h->device = attr.device;
    else if (hipGetDevice(&h->device) != hipSuccess) h->device = -1;
  }
  // rest state g = 0, statistics 0, flags 0 (fill kernels: safe under graph capture)
  hipError_t e = launch_fill_zero(h->gbuf(0), align_up(h->gbytes()), h->stream);
  if (e == hipSuccess) e = launch_fill_zero(h->at<char>(L.stats), L.sponge - L.stats, h->stream);
  if (e == hipSuccess) e = launch_fill_zero(h->at<char>(L.flag), kAlign, h->stream);
  if (e == hipSuccess)
    e = launch_sponge(h->at<float>(L.sponge), desc->nx, desc->periodic_x ? 0 : desc->sponge_cells,
                      desc->sponge_K, desc->sponge_p, h->stream);
  if (e != hipSuccess) {
    const std::string msg = std::string("init kernels: ") + hipGetErrorString(e);
    delete h;
    return fail(nullptr, STGLBM_E_HIP, msg);
  }
  *out = h;
  return STGLBM_OK;
}

int stglbm_set_rans_inlet(stglbm_t h, const stglbm_rans_inlet* in) {
  TraceRange trace("stglbm_set_rans_inlet");
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  if (h->d.periodic_x) return fail(h, STGLBM_E_STATE, "periodic_x lattice has no inlet");
  if (!in || !in->y || !in->U3 || !in->k || !in->omega || !in->R6) return fail(h, STGLBM_E_INVAL, "null RANS input");
  const int n = in->n_rans;
  if (n < 2 || n > h->d.max_rans) return fail(h, STGLBM_E_INVAL, "n_rans out of range");
  if (in->n_modes < 1 || in->n_modes > h->d.max_modes) return fail(h, STGLBM_E_INVAL, "n_modes out of range");
  if (!(in->delta > 0) || !(in->c_x > 0) || !(in->c_t > 0) || !(in->U_b > 0) || !(in->nu_phys > 0) ||
      !(in->C_l > 0) || !(in->C_mu > 0))
    return fail(h, STGLBM_E_INVAL, "delta, c_x, c_t, U_b, nu_phys, C_l, C_mu must be positive");
  if (std::fabs(in->c_x * h->d.ny - 2.0 * in->delta) > 1e-9 * in->delta)
    return fail(h, STGLBM_E_INVAL, "c_x * NY must equal 2 delta");
  if (!(in->y[0] > 0.0) || !(in->y[n - 1] < 2.0 * in->delta)) return fail(h, STGLBM_E_INVAL, "RANS y outside (0, 2 delta)");
  for (int i = 1; i < n; ++i)
    if (!(in->y[i] > in->y[i - 1])) return fail(h, STGLBM_E_INVAL, "RANS y must increase strictly");
  for (int i = 0; i < n; ++i)
    if (!(in->k[i] > 0.0) || !(in->omega[i] > 0.0)) return fail(h, STGLBM_E_INVAL, "k and omega must be positive");
  if (in->n_modes == 1 && !(in->alpha > 0.0)) return fail(h, STGLBM_E_INVAL, "one mode needs alpha > 0");
  int rc = sync_and_check(h);
  if (rc != STGLBM_OK && rc != STGLBM_E_UNSTABLE) return rc;
  // stage the RANS arrays: y[n] U3[n][3] k[n] omega[n] R6[n][6]
  std::vector<double> stage(static_cast<size_t>(n) * 12);
  std::memcpy(stage.data(), in->y, n * sizeof(double));
  std::memcpy(stage.data() + n, in->U3, 3 * n * sizeof(double));
  std::memcpy(stage.data() + 4 * n, in->k, n * sizeof(double));
  std::memcpy(stage.data() + 5 * n, in->omega, n * sizeof(double));
  std::memcpy(stage.data() + 6 * n, in->R6, 6 * n * sizeof(double));
  double* dstage = h->at<double>(h->L.rans);
  HIP_CHECK(h, hipMemcpyAsync(dstage, stage.data(), stage.size() * sizeof(double), hipMemcpyHostToDevice, h->stream),
            "hipMemcpyAsync RANS");
  SetupParams p{};
  p.rans = dstage;
  p.n_rans = n; p.ny = h->d.ny; p.nz = h->d.nz; p.n_modes = in->n_modes;
  p.delta = in->delta; p.nu_phys = in->nu_phys; p.c_x = in->c_x; p.alpha = in->alpha;
  p.C_l = in->C_l; p.C_mu = in->C_mu; p.U_b = in->U_b; p.seed = in->seed;
  p.rows = h->at<double>(h->L.rows);
  p.modes = h->at<double>(h->L.modes);
  p.sqrtq = h->at<double>(h->L.sqrtq);
  p.arow = h->at<double2>(h->L.arow);
  p.bz = h->at<float2>(h->L.bz);
  p.sig = h->at<float4>(h->L.sig);
  p.scalars = h->at<double>(h->L.scalars);
  p.clamps = h->at<int>(h->L.flag) + 1;
  HIP_CHECK(h, launch_inlet_setup(p, h->stream), "inlet setup kernels");
  HIP_CHECK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  double sc[kScalars];
  HIP_CHECK(h, hipMemcpy(sc, p.scalars, sizeof(sc), hipMemcpyDeviceToHost), "hipMemcpy scalars");
  if (in->strict && sc[5] > 0) return fail(h, STGLBM_E_REALIZABILITY, "negative Cholesky radicand (Reynolds stress not realizable)");
  if (!(sc[0] > 0.0) || !std::isfinite(sc[0]) || !std::isfinite(sc[3]))
    return fail(h, STGLBM_E_INVAL, "degenerate inlet length scales");
  h->n_modes = in->n_modes;
  h->c_x = in->c_x; h->c_t = in->c_t; h->U_b = in->U_b; h->L_e = sc[0];
  uint64_t hs = 0xcbf29ce484222325ull;
  hs = fnv1a(hs, stage.data(), stage.size() * sizeof(double));
  const double params[] = {in->delta, in->nu_phys, in->c_x, in->c_t, in->U_b, in->alpha, in->C_l, in->C_mu};
  hs = fnv1a(hs, params, sizeof(params));
  hs = fnv1a(hs, &in->seed, sizeof(in->seed));
  hs = fnv1a(hs, &in->n_modes, sizeof(in->n_modes));
  h->inlet_hash = hs;
  h->inlet_ready = true;
  h->ring_n = 0;
  h->ptab_n = 0;
  return rc;
}

int stglbm_stg_generate(stglbm_t h, int64_t t_step, float* d_u_plane) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  if (h->d.periodic_x || !h->inlet_ready) return fail(h, STGLBM_E_STATE, "no inlet installed");
  if (!d_u_plane) h->ring_n = 0;   // the plane goes to the front of the ring
  return launch_planes(h, t_step, 1, d_u_plane ? d_u_plane : h->at<float>(h->L.ubc));
}

int stglbm_step(stglbm_t h, int32_t n_steps) {
  TraceRange trace("stglbm_step");
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  if (n_steps < 0) return fail(h, STGLBM_E_INVAL, "n_steps < 0");
  if (!h->d.periodic_x && !h->inlet_ready) return fail(h, STGLBM_E_STATE, "set_rans_inlet must precede step");
  for (int32_t s = 0; s < n_steps; ++s) {
    const float* plane = nullptr;
    if (!h->d.periodic_x) {
      if (int rc = ring_plane(h, h->t + 1, &plane)) return rc;
    }
    if (int rc = step_once(h, plane, true, true)) return rc;
  }
  return STGLBM_OK;
}

int stglbm_step_noalloc(stglbm_t h, int32_t n_steps) {
  TraceRange trace("stglbm_step_noalloc");
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  if (n_steps < 0) return fail(h, STGLBM_E_INVAL, "n_steps < 0");
  uint64_t plane_bytes = 0;
  if (!h->d.periodic_x) {
    plane_bytes = h->plane_floats() * sizeof(float);
    if (plane_bytes > kScratchBytes)
      return fail(h, STGLBM_E_INVAL, "step_noalloc: one inlet plane (NY*NZ*3 floats) exceeds the library's " +
                                         std::to_string(kScratchBytes >> 20) + " MiB static scratch");
    if (!h->inlet_ready) return fail(h, STGLBM_E_STATE, "set_rans_inlet must precede step");
  }
  float* planes = nullptr;
  if (int rc = device_scratch(h, reinterpret_cast<void**>(&planes))) return rc;
  // Planes of up to kStgBatch consecutive steps, made one batch at a time into
  // the scratch and used before the next batch overwrites them.
  const int64_t fit = plane_bytes ? static_cast<int64_t>(kScratchBytes / plane_bytes) : kStgBatch;
  const int batch = static_cast<int>(std::min<int64_t>(kStgBatch, fit));
  for (int32_t s = 0; s < n_steps; ++s) {
    const float* plane = nullptr;
    if (!h->d.periodic_x) {
      const int k = s % batch;
      if (k == 0) {
        if (int rc = launch_planes(h, h->t + 1, std::min(batch, n_steps - s), planes, false)) return rc;
      }
      plane = planes + static_cast<uint64_t>(k) * h->plane_floats();
    }
    if (int rc = step_once(h, plane, false)) return rc;
  }
  return STGLBM_OK;
}

int stglbm_set_probes(stglbm_t h, int32_t n, const int32_t* h_xyz, float* d_series, int64_t capacity) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  if (n == 0) {
    h->n_probes = 0;
    h->probe_out = nullptr;
    h->probe_capacity = h->probe_rows = 0;
    return STGLBM_OK;
  }
  if (n < 0 || n > kMaxProbes) return fail(h, STGLBM_E_INVAL, "number of probes must be 0..64");
  if (!h_xyz || !d_series || capacity < 1) return fail(h, STGLBM_E_INVAL, "null probe list or series, or capacity < 1");
  for (int k = 0; k < n; ++k) {
    const int x = h_xyz[3 * k], y = h_xyz[3 * k + 1], z = h_xyz[3 * k + 2];
    if (x < 0 || x >= h->d.nx || y < 0 || y >= h->d.ny || z < 0 || z >= h->d.nz)
      return fail(h, STGLBM_E_INVAL, "probe outside the lattice");
  }
  for (int k = 0; k < n; ++k)
    for (int a = 0; a < 3; ++a) h->probe_xyz[k][a] = h_xyz[3 * k + a];
  h->n_probes = n;
  h->probe_out = d_series;
  h->probe_capacity = capacity;
  h->probe_rows = 0;
  return STGLBM_OK;
}

int stglbm_probe_rows(stglbm_t h, int64_t* rows) {
  if (!h || !rows) return fail(h, STGLBM_E_INVAL, "null handle or output");
  *rows = h->probe_rows;
  return STGLBM_OK;
}

int stglbm_stats_reset(stglbm_t h) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  HIP_CHECK(h, launch_fill_zero(h->at<char>(h->L.stats), h->L.sponge - h->L.stats, h->stream), "stats reset");
  h->n_samples = 0;
  h->sampling = true;
  return STGLBM_OK;
}

int stglbm_stats_stop(stglbm_t h) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  h->sampling = false;
  return STGLBM_OK;
}

int stglbm_get_stats(stglbm_t h, double* h_out, uint64_t n, int64_t* n_samples) {
  TraceRange trace("stglbm_get_stats");
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  const uint64_t bins = static_cast<uint64_t>(h->d.nx) * h->d.ny;
  if (!h_out || n != bins * 9) return fail(h, STGLBM_E_INVAL, "stats buffer must hold NX*NY*9 doubles");
  const int rc = sync_and_check(h);
  const size_t n9 = 9 * bins;
  std::vector<double> raw(n9);
  HIP_CHECK(h, hipMemcpy(raw.data(), h->at<double>(h->L.stats), raw.size() * sizeof(double), hipMemcpyDeviceToHost),
            "hipMemcpy stats");
  std::vector<float> win(static_cast<size_t>(h->L.slots) * n9);
  HIP_CHECK(h, hipMemcpy(win.data(), h->at<float>(h->L.win), win.size() * sizeof(float), hipMemcpyDeviceToHost),
            "hipMemcpy window sums");
  // device layout [slot][k][y][x]; API layout [x][y][k]: the totals plus the
  // current window's slots in order (the fold's own sum, so a later fold gives
  // the same numbers whenever the statistics are read).
  const bool open = h->n_samples % kStatsWindow != 0;
  for (int x = 0; x < h->d.nx; ++x)
    for (int y = 0; y < h->d.ny; ++y)
      for (int k = 0; k < 9; ++k) {
        const size_t e = static_cast<size_t>(k) * bins + static_cast<size_t>(y) * h->d.nx + x;
        double v = raw[e];
        if (open)
          for (int s = 0; s < h->L.slots; ++s) v += static_cast<double>(win[static_cast<size_t>(s) * n9 + e]);
        h_out[(static_cast<size_t>(x) * h->d.ny + y) * 9 + k] = v;
      }
  if (n_samples) *n_samples = h->n_samples;
  return rc;
}

int stglbm_get_f(stglbm_t h, double* h_out, uint64_t n) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  const uint64_t total = static_cast<uint64_t>(h->q()) * h->cells();
  if (!h_out || n != total) return fail(h, STGLBM_E_INVAL, "f buffer must hold Q*NX*NY*NZ doubles");
  const int rc = sync_and_check(h);
  double* stage = static_cast<double*>(h->gbuf(1 - h->cur));
  const uint64_t chunk = h->gbytes() / sizeof(double);
  for (uint64_t off = 0; off < total; off += chunk) {
    const uint64_t cnt = std::min<uint64_t>(chunk, total - off);
    HIP_CHECK(h, launch_export_f(h->gbuf(h->cur), h->d.store, h->q(), off, cnt, h->d.nz,
                                 static_cast<long long>(h->d.nx) * h->d.ny, stage, h->stream), "export kernel");
    HIP_CHECK(h, hipMemcpyAsync(h_out + off, stage, cnt * sizeof(double), hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync f");
    HIP_CHECK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  }
  return rc;
}

int stglbm_get_f_planes(stglbm_t h, int32_t x0, int32_t x1, double* h_out, uint64_t n) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  if (x0 < 0 || x1 > h->d.nx || x1 <= x0) return fail(h, STGLBM_E_INVAL, "need 0 <= x0 < x1 <= NX");
  const uint64_t total = static_cast<uint64_t>(h->q()) * h->d.nz * h->d.ny * (x1 - x0);
  if (!h_out || n != total) return fail(h, STGLBM_E_INVAL, "buffer must hold Q*NZ*NY*(x1-x0) doubles");
  const int rc = sync_and_check(h);
  double* stage = static_cast<double*>(h->gbuf(1 - h->cur));
  const uint64_t chunk = h->gbytes() / sizeof(double);   // the inactive buffer stages one chunk at a time
  for (uint64_t off = 0; off < total; off += chunk) {
    const uint64_t cnt = std::min<uint64_t>(chunk, total - off);
    HIP_CHECK(h, launch_export_planes(h->gbuf(h->cur), h->d.store, h->q(), h->d.nx, h->d.ny, h->d.nz, x0, x1,
                                      static_cast<long long>(off), static_cast<long long>(cnt), stage, h->stream),
              "export kernel");
    HIP_CHECK(h, hipMemcpyAsync(h_out + off, stage, cnt * sizeof(double), hipMemcpyDeviceToHost, h->stream),
              "hipMemcpyAsync f");
    HIP_CHECK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  }
  return rc;
}

int stglbm_state_view(stglbm_t h, void** d_g, uint64_t* bytes) {
  if (!h || !d_g || !bytes) return fail(h, STGLBM_E_INVAL, "null argument");
  *d_g = h->gbuf(h->cur);
  *bytes = h->gbytes();
  return STGLBM_OK;
}

int stglbm_set_f(stglbm_t h, const double* h_in, uint64_t n) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  const uint64_t total = static_cast<uint64_t>(h->q()) * h->cells();
  if (!h_in || n != total) return fail(h, STGLBM_E_INVAL, "f buffer must hold Q*NX*NY*NZ doubles");
  const int rc = sync_and_check(h);
  if (rc != STGLBM_OK && rc != STGLBM_E_UNSTABLE) return rc;
  double* stage = static_cast<double*>(h->gbuf(1 - h->cur));
  const uint64_t chunk = h->gbytes() / sizeof(double);
  for (uint64_t off = 0; off < total; off += chunk) {
    const uint64_t cnt = std::min<uint64_t>(chunk, total - off);
    HIP_CHECK(h, hipMemcpyAsync(stage, h_in + off, cnt * sizeof(double), hipMemcpyHostToDevice, h->stream), "hipMemcpyAsync f");
    HIP_CHECK(h, launch_import_f(stage, h->d.store, h->q(), off, cnt, h->d.nz,
                                 static_cast<long long>(h->d.nx) * h->d.ny, h->gbuf(h->cur), h->stream), "import kernel");
    HIP_CHECK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  }
  HIP_CHECK(h, launch_fill_zero(h->at<char>(h->L.flag), kAlign, h->stream), "flag reset");
  HIP_CHECK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  return STGLBM_OK;
}

namespace {

int set_equilibrium_scaled(stglbm_t h, const double* h_u, uint64_t n, double scale) {
  const uint64_t total = 3ull * h->cells();
  if (!h_u || n != total) return fail(h, STGLBM_E_INVAL, "u buffer must hold 3*NX*NY*NZ doubles");
  const int rc = sync_and_check(h);
  if (rc != STGLBM_OK && rc != STGLBM_E_UNSTABLE) return rc;
  // staged in the idle distribution buffer (Q s >= 30 >= 24 bytes per cell for every set and store)
  double* stage = static_cast<double*>(h->gbuf(1 - h->cur));
  HIP_CHECK(h, hipMemcpyAsync(stage, h_u, total * sizeof(double), hipMemcpyHostToDevice, h->stream), "hipMemcpyAsync u");
  HIP_CHECK(h, launch_equilibrium(stage, scale, h->d.store, h->q(), h->d.nx, h->d.ny, h->d.nz, h->gbuf(h->cur),
                                  h->stream),
            "equilibrium kernel");
  HIP_CHECK(h, launch_fill_zero(h->at<char>(h->L.flag), kAlign, h->stream), "flag reset");
  HIP_CHECK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  return STGLBM_OK;
}

}  // namespace

int stglbm_set_equilibrium(stglbm_t h, const double* h_u, uint64_t n) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  return set_equilibrium_scaled(h, h_u, n, 1.0);
}

int stglbm_set_equilibrium_physical(stglbm_t h, const double* h_u, uint64_t n, double c_x, double c_t) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  if (!(c_x > 0.0) || !(c_t > 0.0) || !std::isfinite(c_x) || !std::isfinite(c_t))
    return fail(h, STGLBM_E_INVAL, "c_x and c_t must be positive");
  return set_equilibrium_scaled(h, h_u, n, c_t / c_x);
}

static int copy_out(stglbm_t h, uint64_t off, uint64_t bytes, double* out) {
  const int rc = sync_and_check(h);
  HIP_CHECK(h, hipMemcpy(out, h->ws + off, bytes, hipMemcpyDeviceToHost), "hipMemcpy");
  return rc;
}

int stglbm_get_modes(stglbm_t h, double* h_out, uint64_t n) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  if (!h->inlet_ready) return fail(h, STGLBM_E_STATE, "no inlet installed");
  if (!h_out || n != static_cast<uint64_t>(h->n_modes) * kModeFields) return fail(h, STGLBM_E_INVAL, "modes buffer must hold N*8 doubles");
  return copy_out(h, h->L.modes, n * sizeof(double), h_out);
}

int stglbm_get_inlet_rows(stglbm_t h, double* h_out, uint64_t n) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  if (!h->inlet_ready) return fail(h, STGLBM_E_STATE, "no inlet installed");
  if (!h_out || n != static_cast<uint64_t>(h->d.ny) * kRowFields) return fail(h, STGLBM_E_INVAL, "rows buffer must hold NY*18 doubles");
  return copy_out(h, h->L.rows, n * sizeof(double), h_out);
}

int stglbm_get_inlet_scalars(stglbm_t h, double* h_out, uint64_t n) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  if (!h->inlet_ready) return fail(h, STGLBM_E_STATE, "no inlet installed");
  if (!h_out || n != kScalars) return fail(h, STGLBM_E_INVAL, "scalars buffer must hold 8 doubles");
  return copy_out(h, h->L.scalars, n * sizeof(double), h_out);
}

int stglbm_get_sqrtq(stglbm_t h, double* h_out, uint64_t n) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  if (!h->inlet_ready) return fail(h, STGLBM_E_STATE, "no inlet installed");
  if (!h_out || n != static_cast<uint64_t>(h->d.ny) * h->n_modes) return fail(h, STGLBM_E_INVAL, "sqrtq buffer must hold NY*N doubles");
  return copy_out(h, h->L.sqrtq, n * sizeof(double), h_out);
}

int stglbm_get_step(stglbm_t h, int64_t* t) {
  if (!h || !t) return fail(h, STGLBM_E_INVAL, "null argument");
  *t = h->t;
  return STGLBM_OK;
}

int stglbm_set_stream(stglbm_t h, void* hip_stream) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  HIP_CHECK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->ring_n = 0;   // planes made on the old stream are not ordered before work on the new one
  h->ptab_n = 0;
  return STGLBM_OK;
}

int stglbm_sync(stglbm_t h) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  return sync_and_check(h);
}

int stglbm_checkpoint_size(stglbm_t h, uint64_t* bytes) {
  if (!h || !bytes) return fail(h, STGLBM_E_INVAL, "null argument");
  *bytes = sizeof(CkptHeader) + h->gbytes() + (h->L.sponge - h->L.stats);
  return STGLBM_OK;
}

int stglbm_checkpoint(stglbm_t h, void* h_buf, uint64_t n) {
  TraceRange trace("stglbm_checkpoint");
  uint64_t need = 0;
  if (int rc = stglbm_checkpoint_size(h, &need)) return rc;
  if (!h_buf || n < need) return fail(h, STGLBM_E_INVAL, "checkpoint buffer too small");
  const int rc = sync_and_check(h);
  if (rc != STGLBM_OK) return rc;
  CkptHeader hd{};
  hd.magic = kCkptMagic; hd.version = kCkptVersion;
  hd.nx = h->d.nx; hd.ny = h->d.ny; hd.nz = h->d.nz; hd.store = h->d.store; hd.periodic_x = h->d.periodic_x;
  hd.slots = h->L.slots; hd.inlet_hash = h->inlet_hash; hd.t = h->t; hd.n_samples = h->n_samples;
  hd.sampling = h->sampling ? 1 : 0; hd.n_modes = h->n_modes;
  hd.g_bytes = h->gbytes(); hd.stats_bytes = h->L.sponge - h->L.stats;
  hd.q = h->q(); hd.collision = h->d.collision;
  char* out = static_cast<char*>(h_buf);
  std::memcpy(out, &hd, sizeof(hd));
  HIP_CHECK(h, hipMemcpy(out + sizeof(hd), h->gbuf(h->cur), hd.g_bytes, hipMemcpyDeviceToHost), "hipMemcpy g");
  HIP_CHECK(h, hipMemcpy(out + sizeof(hd) + hd.g_bytes, h->ws + h->L.stats, hd.stats_bytes, hipMemcpyDeviceToHost), "hipMemcpy stats");
  return STGLBM_OK;
}

int stglbm_restore(stglbm_t h, const void* h_buf, uint64_t n) {
  TraceRange trace("stglbm_restore");
  if (!h || !h_buf) return fail(h, STGLBM_E_INVAL, "null argument");
  if (n < sizeof(CkptHeader)) return fail(h, STGLBM_E_INVAL, "checkpoint too short");
  CkptHeader hd;
  std::memcpy(&hd, h_buf, sizeof(hd));
  if (hd.magic != kCkptMagic || hd.version != kCkptVersion) return fail(h, STGLBM_E_INVAL, "not a checkpoint of this library");
  if (hd.nx != h->d.nx || hd.ny != h->d.ny || hd.nz != h->d.nz || hd.store != h->d.store ||
      hd.periodic_x != h->d.periodic_x || hd.slots != h->L.slots || hd.q != h->q() ||
      hd.collision != h->d.collision)
    return fail(h, STGLBM_E_INVAL, "checkpoint lattice differs from the handle's");
  if (!h->d.periodic_x && (!h->inlet_ready || hd.inlet_hash != h->inlet_hash || hd.n_modes != h->n_modes))
    return fail(h, STGLBM_E_STATE, "install the same inlet (set_rans_inlet) before restoring");
  if (n < sizeof(hd) + hd.g_bytes + hd.stats_bytes || hd.g_bytes != h->gbytes() ||
      hd.stats_bytes != h->L.sponge - h->L.stats)
    return fail(h, STGLBM_E_INVAL, "checkpoint size mismatch");
  HIP_CHECK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  const char* in = static_cast<const char*>(h_buf);
  HIP_CHECK(h, hipMemcpy(h->gbuf(h->cur), in + sizeof(hd), hd.g_bytes, hipMemcpyHostToDevice), "hipMemcpy g");
  HIP_CHECK(h, hipMemcpy(h->ws + h->L.stats, in + sizeof(hd) + hd.g_bytes, hd.stats_bytes, hipMemcpyHostToDevice), "hipMemcpy stats");
  HIP_CHECK(h, launch_fill_zero(h->at<char>(h->L.flag), kAlign, h->stream), "flag reset");
  HIP_CHECK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  h->t = hd.t;
  h->ring_n = 0;
  h->ptab_n = 0;
  h->n_samples = hd.n_samples;
  h->sampling = hd.sampling != 0;
  return STGLBM_OK;
}

int stglbm_profile(stglbm_t h, int32_t enable) {
  if (!h) return fail(nullptr, STGLBM_E_INVAL, "null handle");
  if (enable < 0) return fail(h, STGLBM_E_INVAL, "profile: enable must be >= 0");
  h->prof = enable != 0;
  h->prof_every = enable > 0 ? enable : 1;
  h->prof_count = 0;
  return STGLBM_OK;
}

int stglbm_profile_read(stglbm_t h, double* out, uint64_t n) {
  if (!h || !out || n < 5) return fail(h, STGLBM_E_INVAL, "profile buffer must hold 5 doubles");
  HIP_CHECK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  double ms_step = 0.0, ms_stg = 0.0;
  for (size_t i = 0; i < h->n_step; ++i) {
    float ms = 0.f;
    HIP_CHECK(h, hipEventElapsedTime(&ms, h->ev_step[2 * i], h->ev_step[2 * i + 1]), "hipEventElapsedTime");
    ms_step += ms;
  }
  for (size_t i = 0; i < h->n_stg; ++i) {
    float ms = 0.f;
    HIP_CHECK(h, hipEventElapsedTime(&ms, h->ev_stg[2 * i], h->ev_stg[2 * i + 1]), "hipEventElapsedTime");
    ms_stg += ms;
  }
  out[0] = ms_step; out[1] = static_cast<double>(h->n_step);
  out[2] = ms_stg; out[3] = static_cast<double>(h->n_planes); out[4] = static_cast<double>(h->n_stg);
  if (n >= 6) out[5] = static_cast<double>(h->n_tail_planes);
  h->n_step = h->n_stg = h->n_planes = h->n_tail_planes = 0;
  return STGLBM_OK;
}

int stglbm_copy_probe(const void* d_src, void* d_dst, uint64_t bytes, void* hip_stream) {
  if (!d_src || !d_dst || bytes % 16) return fail(nullptr, STGLBM_E_INVAL, "copy_probe needs non-null buffers and bytes % 16 == 0");
  const hipError_t e = launch_copy(d_src, d_dst, bytes, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(nullptr, STGLBM_E_HIP, std::string("copy kernel: ") + hipGetErrorString(e));
  return STGLBM_OK;
}

int stglbm_bandwidth_probe(const void* d_src, void* d_dst, uint64_t bytes, int32_t mode, void* hip_stream) {
  if ((mode != 3 && !d_src) || (mode != 2 && !d_dst) || bytes % 16 || mode < 0 || mode > 3)
    return fail(nullptr, STGLBM_E_INVAL, "bandwidth_probe needs mode 0..3, the buffers it uses and bytes % 16 == 0");
  const hipError_t e = launch_bandwidth_probe(d_src, d_dst, bytes, mode, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(nullptr, STGLBM_E_HIP, std::string("bandwidth probe: ") + hipGetErrorString(e));
  return STGLBM_OK;
}

int stglbm_destroy(stglbm_t h) {
  if (!h) return STGLBM_OK;
  if (h->stream || true) (void)hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->ev_step) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->ev_stg) (void)hipEventDestroy(e);
  delete h;
  return STGLBM_OK;
}

const char* stglbm_last_error(stglbm_t h) { return h ? h->err.c_str() : g_lib_error.c_str(); }

}  // extern "C"
