// Internal declarations shared by the kernels and the C ABI of libstglbm.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace stglbm {

constexpr int kRowFields = 18;      // U(3) k omega R(6) a(6) l_e
constexpr int kModeFields = 8;      // k, d(3), sigma(3), phi
constexpr int kScalars = 8;         // L_e k_min k_max alpha k_cut clamps U_b N
constexpr int kMaxWavesPerBlock = 8; // step kernel: waves along x times waves along z
constexpr int kMaxWavesWide = 16;    // FP32 statistics launches of D3Q15 / D3Q19, one cell per lane
constexpr int kStgInFlight = 8;     // spanwise phasor loads in flight per wave of the plane kernel
constexpr int kStgWaves = 8;        // waves per STG block, each summing 1/8 of the modes
constexpr int kStgBatch = 16;       // inlet planes per plane-kernel launch; ring of planes made ahead
constexpr int kStgTailRows = 4;     // rows per plane block of a 16-bit statistics launch
constexpr int kStgTailInFlight = 8; // spanwise phasor loads in flight per wave there

// Waves per block a step-kernel instantiation is built for.  The FP32
// statistics launches of D3Q15 and D3Q19 with one cell per lane fit 16 waves
// in a CU's registers (at most 128 VGPRs) and run two z waves of a whole row
// per block; every other instantiation stays at 8 (D3Q27 and wider lanes need
// more registers).
constexpr int step_max_waves(int store_bytes, int q, int vec, bool stats) {
  return (stats && store_bytes == 4 && q <= 19 && vec == 1) ? kMaxWavesWide : kMaxWavesPerBlock;
}

// Flag bits written by the kernels into the handle's status word.
constexpr int kFlagDensity = 1;     // |rho - 1| >= 0.5 or NaN in the step kernel
constexpr int kFlagInletMach = 2;   // |u_bc,x| >= 0.3 c_s at an inlet node

// STG inlet planes: a launch of the plane kernel, or the trailing blocks of a
// stream-collide launch.
struct StgParams {
  const double* modes;      // [N][8]
  const double2* arow;      // [N][NY] sqrt 6 sqrt(q^n) exp(i (k^n d^n_y y_j + phi^n))
  const float2* bz;         // [N][NZ] spanwise phasors exp(i k d_z z)
  const float4* sig;        // [N] sigma^n in FP32 (x, y, z, 0)
  const double* rows;       // [NY][18]
  float* out;               // n_planes planes [NY][NZ][3], one after the other
  float2* ptab;             // row phasors of kStgBatch steps: [slot][N][ptab_rows] FP32, rows past NY zero
  int ptab_rows;            // NY rounded up to a multiple of 8
  int pslot[kStgBatch];     // table slot of each plane
  int ny, nz, n_modes;
  int n_planes;             // 1 .. kStgBatch consecutive steps
  double c_x;               // lattice spacing (m)
  double conv;              // c_t / c_x
  double tphase[kStgBatch]; // 2 pi (x_in - U_b t) / L_e for the step of each plane
};

// Fused stream-collide pass, one launch per time step.
constexpr int kMaxZChunks = 64;     // z chunks of a statistics launch with unequal chunks

struct StepParams {
  const void* gin;          // g at step n, [NZ][Q][NY][NX] in the store type
  void* gout;               // g at step n+1
  long long plane2d;        // NX*NY: one population of one z slice
  int nx, ny, nz;
  int q;                    // velocity set: 15, 19 or 27 populations
  int collision;            // 0 regularized, 1 plain BGK
  int vec;                  // consecutive x cells per lane (1, 2 or 4)
  int nxt;                  // number of x tiles of 64 * vec cells
  int wx, wz;               // block = wx waves along x times wz waves along z
  int nxg;                  // x-tile groups per row: ceil(nxt / wx)
  int slots;                // spanwise blocks per (x group, y); statistics slots
  int lw;                   // spanwise cells per wave
  int zstep;                // z distance between a wave's rows: slots * wz (interleaved) or wz (chunked)
  int nblocks;
  int remap;                // 1: the blocks of a row share an XCD (nxg > 1, nblocks % (8 nxg) == 0)
  int lockstep;             // statistics launches with wz = 1: a barrier per z row
  int periodic_x;
  int has_force;
  float tau0, tau0_sq;      // tau0 and tau0^2 (rounded from FP64)
  float s0;                 // tau0 - 1/2 (rounded from FP64)
  float c18;                // 18 sqrt(2) Cs^2
  float fx, fy, fz;         // Guo acceleration
  float rho_out_m1;         // rho_out - 1
  float inv_rho_out;        // 1/rho_out
  float mach_limit;         // inlet guard: |u_bc,x| < 0.3 c_s
  const float* sponge;      // [NX] viscosity multipliers (all 1 if no sponge)
  const float* ubc;         // [NY][NZ][3] inlet velocity of this step (lattice units)
  double* stats;            // [9][NY][NX] FP64 totals of the closed windows (not written by the kernel)
  float* win;               // [slots][9][NY][NX] FP32 sums of the current window
  int win_first;            // first sampled step of a window (store, not add)
  int* flag;
  // Trailing blocks (blockIdx.x >= nblocks) make one inlet plane of a later
  // step while the launch's last lattice blocks finish (0: none).
  int stg_blocks;
  int stg_zb;               // blocks of 64 spanwise nodes per plane row group
  StgParams stg;            // that plane: out, tphase[0]
  // Statistics launches with unequal z chunks (zsched = 1): the blocks of slot
  // s take z rows zbeg[s] .. zbeg[s + 1] - 1 (multiples of wz rows)
  int zsched;
  int zbeg[kMaxZChunks + 1];
  // FP32 D3Q19 regularized statistics launches: the kernel built with the
  // max-ilp machine scheduler instead of the default one
  int f32_ilp;
};

// Statistics: every launch adds its per-slot sums to FP32 window sums; after kStatsWindow sampled steps (counted from stats_reset) they
// are folded, in slot order, into the FP64 totals [9][NY][NX].
constexpr int kStatsWindow = 16;

// Velocity probes: after a step, u at up to kMaxProbes cells of the new state.
constexpr int kMaxProbes = 64;
struct ProbeParams {
  const void* g;            // state just written, [NZ][Q][NY][NX]
  long long plane2d;        // NX*NY
  int q, nx, n;
  double fx, fy, fz;        // Guo acceleration (u = (sum c f - F/2) / rho)
  int xyz[kMaxProbes][3];
  float* out;               // this step's row of the series: [n][3]
};

// One-off inlet precompute.
struct SetupParams {
  const double* rans;       // staging: y[n] U3[n][3] k[n] omega[n] R6[n][6]
  int n_rans, ny, nz, n_modes;
  double delta, nu_phys, c_x, alpha, C_l, C_mu, U_b;
  unsigned long long seed;
  double* rows;             // [NY][18]
  double* modes;            // [N][8]
  double* sqrtq;            // [NY][N]
  double2* arow;            // [N][NY] time-independent row phasors of the plane kernel
  float2* bz;               // [N][NZ]
  float4* sig;              // [N]
  double* scalars;          // [8]
  int* clamps;
};

hipError_t launch_step(const StepParams& p, int store, bool stats, hipStream_t s);
hipError_t launch_step_variant(const StepParams& p, int store, bool stats, hipStream_t s);
// Row phasors of p.n_planes steps into the table slots p.pslot (before any
// plane kernel or trailing block that reads them).
hipError_t launch_stg_time_phase(const StgParams& p, hipStream_t s);
hipError_t launch_stg(const StgParams& p, hipStream_t s);
hipError_t launch_inlet_setup(const SetupParams& p, hipStream_t s);
hipError_t launch_fill_zero(void* ptr, unsigned long long bytes, hipStream_t s);
// out[e] = (add ? out[e] : 0) + sum_s d[s n + e] (s < nd) + sum_s f[s n + e] (s < nf),
// FP64, in that order, for e < n.
hipError_t launch_stats_sum(const double* d, int nd, const float* f, int nf, long long n, double* out, bool add,
                            hipStream_t s);
hipError_t launch_sponge(float* sponge, int nx, int cells, double K, double p, hipStream_t s);
// Public order [Q][NZ][NY][NX] <-> stored order [NZ][Q][NY][NX].
hipError_t launch_export_f(const void* g, int store, int q, long long offset, long long count, int nz,
                           long long plane2d, double* out, hipStream_t s);
hipError_t launch_export_planes(const void* g, int store, int q, int nx, int ny, int nz, int x0, int x1,
                                long long offset, long long count, double* out, hipStream_t s);
hipError_t launch_import_f(const double* f, int store, int q, long long offset, long long count, int nz,
                           long long plane2d, void* g, hipStream_t s);
// f_eq(1, scale * u), u component-major [3][NZ][NY][NX] (scale: unit conversion, 1 for lattice units).
hipError_t launch_equilibrium(const double* u, double scale, int store, int q, int nx, int ny, int nz, void* g,
                              hipStream_t s);
hipError_t launch_probes(const ProbeParams& p, int store, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, unsigned long long bytes, hipStream_t s);
// mode 0: the plain copy; 1: copy with 4 x 16 B loads in flight per lane and non-temporal
// stores; 2: read-only sweep of src (dst unchanged); 3: write-only fill of dst.
hipError_t launch_bandwidth_probe(const void* src, void* dst, unsigned long long bytes, int mode, hipStream_t s);

}  // namespace stglbm
