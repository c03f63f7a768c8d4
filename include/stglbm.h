/*
 * stglbm.h -- C ABI of the STG-LBM hot path on one MI355X (gfx950).
 *
 * The library advances a regularized D3Q19 lattice-Boltzmann large-eddy
 * simulation (Smagorinsky eddy viscosity) of a 3-D channel whose inlet plane
 * is fed by a synthetic turbulence generator (STG) built from RANS data, and
 * whose outlet is a regularized pressure boundary with a sponge zone before
 * it.  Method: Xue, Yao & Davidson, "Synthetic turbulence generator for
 * lattice Boltzmann method at the interface between RANS and LES"
 * (Methodology section; STG section; Algorithm 1; Numerical setup section).
 *
 * Geometry.  Lattice NX x NY x NZ.  x is streamwise: inlet plane x = 0,
 * outlet plane x = NX-1 (or periodic).  y is wall-normal with halfway
 * bounce-back walls at y = -1/2 and y = NY-1/2.  z is spanwise and periodic.
 *
 * Memory.  The caller owns all device memory: init_lattice carves one
 * caller-provided workspace of stglbm_footprint() bytes and the library
 * never allocates device memory.  The caller also owns the HIP stream
 * (hipStream_t passed as void*); every kernel of a handle runs on it.
 * Host arrays passed in are only read during the call.
 *
 * Distributions.  Stored as deviations g_i = f_i - w_i in two buffers
 * (read one, write the other, swapped every step), as FP32, FP16 or BF16
 * (round to nearest even); arithmetic is FP32, statistics FP64.
 * Device layout [NZ][Q][NY][NX] (each z slice holds all Q populations, Q = 19
 * unless the descriptor selects D3Q15 or D3Q27;
 * x fastest); the host-side arrays of get_f/set_f/get_f_planes are
 * [Q][NZ][NY][NX].  D3Q19 population order: rest;
 * +x, -x, +y, -y, +z, -z; (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0),
 * (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1),
 * (0,-1,1).
 *
 * Errors.  Every call returns an int: STGLBM_OK (0) or a negative code;
 * stglbm_last_error() gives the message.  stglbm_step is asynchronous: an
 * instability detected on the device (density deviation outside
 * (-0.5, 0.5), NaN, or |u_bc,x| >= 0.3 c_s at an inlet node) is reported as
 * STGLBM_E_UNSTABLE by the next synchronizing call (get_*, set_*,
 * checkpoint, sync).  A handle is not thread-safe; distinct handles are
 * independent and may run concurrently on different streams.
 */
#ifndef STGLBM_H
#define STGLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stglbm_ctx* stglbm_t;

enum stglbm_status {
  STGLBM_OK = 0,
  STGLBM_E_INVAL = -1,          /* bad argument, size or descriptor            */
  STGLBM_E_NOMEM = -2,          /* workspace smaller than stglbm_footprint()   */
  STGLBM_E_HIP = -3,            /* a HIP runtime call or kernel launch failed  */
  STGLBM_E_STATE = -4,          /* call out of order (e.g. step before inlet)  */
  STGLBM_E_UNSTABLE = -5,       /* device flagged an instability               */
  STGLBM_E_REALIZABILITY = -6   /* Reynolds stress not positive semi-definite  */
};

enum stglbm_store { STGLBM_F32 = 0, STGLBM_F16 = 1, STGLBM_BF16 = 2 };

/* Lattice description (all lattice units).  Field order and padding are
 * part of the ABI. */
typedef struct {
  int32_t nx, ny, nz;       /* lattice size; nx, ny >= 2, nz >= 1, cells < 2^31      */
  int32_t store;            /* enum stglbm_store                                     */
  int32_t periodic_x;       /* 1: x periodic, no inlet/outlet/sponge                  */
  int32_t sponge_cells;     /* L_s: sponge over x in [NX-1-L_s, NX-1]; 0 = off        */
  int32_t max_modes;        /* capacity of the STG mode tables (0 if periodic_x)      */
  int32_t max_rans;         /* capacity of the RANS input staging (0 if periodic_x)   */
  int32_t velocity_set;     /* 19 (or 0): D3Q19, the method's set; 15: D3Q15; 27:
                               D3Q27 (the boundary treatment carries over, Numerical
                               method).  Population order: rest, then opposite pairs
                               (i, i+1), i odd: the 6 axes, then for D3Q19/D3Q27 the
                               12 face diagonals, then for D3Q15/D3Q27 the 8 corners
                               (1,1,1), (-1,-1,-1), (1,1,-1), (-1,-1,1), (1,-1,1),
                               (-1,1,-1), (-1,1,1), (1,-1,-1)                          */
  int32_t collision;        /* 0: regularized BGK bulk (the default configuration);
                               1: plain BGK bulk, eq. lbe                              */
  double nu_lb;             /* molecular viscosity; tau0 = 1/2 + 3 nu (eq. lbe-nu)    */
  double cs_smag;           /* Smagorinsky Cs; the paper's C = Cs^2 (eq. smogrinsky)  */
  double force[3];          /* Guo volume acceleration (eq. bodyforce)               */
  double rho_out;           /* outlet density                                         */
  double sponge_K;          /* eq. sponge_visco: nu (1 + K s^p)                       */
  double sponge_p;
} stglbm_lattice_desc;

/* RANS data at the interface and STG parameters (Algorithm 1, RANS section
 * step 2 and LBM section steps 1-4).  Physical units (m, s). */
typedef struct {
  int32_t n_rans;           /* number of RANS points (FV cell centres)               */
  int32_t n_modes;          /* N Fourier modes (eq. aux_vec), 1 <= N <= max_modes     */
  const double* y;          /* [n_rans] strictly increasing, inside (0, 2 delta)     */
  const double* U3;         /* [n_rans][3] mean velocity                             */
  const double* k;          /* [n_rans] turbulent kinetic energy                     */
  const double* omega;      /* [n_rans] specific dissipation rate                    */
  const double* R6;         /* [n_rans][6] R11, R22, R33, R12, R13, R23              */
  double delta;             /* channel half-height; the lattice spans 2 delta in y   */
  double nu_phys;           /* kinematic viscosity (for the Kolmogorov scale)        */
  double c_x;               /* length conversion (eq. c_factor): 2 delta / NY         */
  double c_t;               /* time conversion (eq. c_factor)                        */
  double U_b;               /* RANS bulk velocity used in the pseudo-position (eq. psu) */
  double alpha;             /* k^n = k_min (1+alpha)^(n-1); <= 0: chosen so k^N = k_max */
  uint64_t seed;            /* SplitMix64 seed of the mode draw                      */
  double C_l;               /* l_e = min(2 d_w, C_l l_t), 3.0                        */
  double C_mu;              /* l_t = sqrt(k)/(C_mu omega), 0.09                      */
  int32_t strict;           /* 1: a negative Cholesky radicand is an error            */
  int32_t reserved;
} stglbm_rans_inlet;

/* Library version (major*10000 + minor*100 + patch). */
int stglbm_version(void);

/* Message of a status code. */
const char* stglbm_status_string(int status);

/* Unit conversion for a channel (Numerical setup section; eqs. c_factor,
 * u_transfer, lbe-nu): c_x = 2 delta / NY, c_t = u_b_lb c_x / U_b,
 * nu_lb = nu_phys c_t / c_x^2.  Host arithmetic in FP64. */
int stglbm_derive_units(double delta, int32_t ny, double u_b_lb, double U_b, double nu_phys,
                        double* c_x, double* c_t, double* nu_lb);

/* Guo volume acceleration in lattice units from a physical one (m/s^2):
 * F = a c_t^2 / c_x, the acceleration unit of eq. c_factor (the paper's
 * periodic reference channel: 1 m/s^2 becomes 3.086e-8 at its resolution).
 * a_phys and force_lb are host arrays of 3 doubles.  FP64 host arithmetic.
 * E_INVAL for null arrays or non-positive c_x, c_t. */
int stglbm_acceleration_to_lattice(double c_x, double c_t, const double* a_phys, double* force_lb);

/* Bytes of device workspace a lattice needs (256-byte aligned pieces). */
int stglbm_footprint(const stglbm_lattice_desc* desc, uint64_t* bytes);

/* Create a handle on a caller-owned workspace (>= footprint bytes, 256-byte
 * aligned) and stream.  The state becomes rest, f_i = w_i (g = 0; Results
 * section), the step counter 0, the statistics empty.  Launches work on the
 * stream and returns without waiting. */
int stglbm_init_lattice(const stglbm_lattice_desc* desc, void* d_workspace, uint64_t ws_bytes,
                        void* hip_stream, stglbm_t* out);

/* Install the RANS inlet and precompute the STG tables on the device in FP64
 * (Algorithm 1, LBM steps 1-4): interpolation to the lattice rows, Cholesky
 * factor (eq. cholesky), l_t, l_e, l_cut (eq. lcut), wavenumbers, the
 * modified von Karman weights q^n (eq. qn), the SplitMix64 mode draw (eq. dn)
 * and the spanwise phase table.  Synchronizes the stream.
 * E_STATE if periodic_x; E_INVAL on bad sizes; E_REALIZABILITY if strict and
 * a radicand was negative (otherwise it is clamped to 0 and counted). */
int stglbm_set_rans_inlet(stglbm_t h, const stglbm_rans_inlet* in);

/* Inlet velocity plane at step index t_step (the state being produced),
 * eqs. aux_vec, psu, v_fluc, u_phys, u_transfer, in lattice units.
 * Writes [NY][NZ][3] FP32 to d_u_plane (device) if non-null, else to the
 * handle's own inlet buffer (the planes stglbm_step made ahead are then
 * made again when needed).  Asynchronous on the stream.  The inlet guard
 * |u_x| < 0.3 c_s is applied by stglbm_step, to the planes it uses. */
int stglbm_stg_generate(stglbm_t h, int64_t t_step, float* d_u_plane);

/* Advance n_steps time steps (Algorithm 1, steps 5-12): for each step the STG
 * plane at t+1 (one launch makes the planes of 16 consecutive steps, kept until
 * used, also by later calls; while a 16-bit store samples statistics, each
 * step launch then makes the plane two steps ahead in trailing blocks of its
 * own, bit-identical to the STG launch's), then one fused pass: pull streaming with
 * bounce-back walls and spanwise wrap, regularized inlet rebuild (eqs. f_i ..
 * bc_eq) behind the guard |u_x| < 0.3 c_s, regularized pressure outlet,
 * moments, Smagorinsky tau_eff (eqs. strain, tau_eff), the sponge (eq.
 * sponge_visco), regularized BGK collision with Guo force, and, while
 * sampling, FP64 statistics.  Asynchronous on the stream. */
int stglbm_step(stglbm_t h, int32_t n_steps);

/* stglbm_step for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and results, bit for bit, but the inlet planes computed ahead of the
 * steps are staged in a static device array of the library (16 MiB, one copy
 * per GPU, held until the process ends) instead of the handle's plane ring,
 * and no profiling events are recorded for these steps.  It calls no
 * allocating routine.  The planes of up to 16 steps are made per STG launch
 * (fewer if they would not fit) and used within the same call; nothing is
 * carried between calls, and the handle's own ring is left as it was.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (two handles on two streams at once) race and must be serialized by
 * the caller.  Errors: E_INVAL if one inlet plane (NY*NZ*3 floats) exceeds
 * the 16 MiB array, or n_steps < 0; E_STATE before set_rans_inlet on an
 * inlet channel; E_HIP if the array's device address cannot be obtained.
 * Periodic-x lattices need no planes and step exactly as stglbm_step. */
int stglbm_step_noalloc(stglbm_t h, int32_t n_steps);

/* Zero the statistics and start sampling every subsequent step. */
int stglbm_stats_reset(stglbm_t h);
/* Stop sampling (statistics are kept). */
int stglbm_stats_stop(stglbm_t h);

/* Statistics sums [NX][NY][9] FP64 over z and sampled steps of
 * u, v, w, uu, vv, ww, uv, uw, vw (velocity of each cell after streaming and
 * any boundary rebuild, the one the collision used; eq. v_rms inputs), and
 * the number of sampled steps.  Synchronizes. n = NX*NY*9. */
int stglbm_get_stats(stglbm_t h, double* h_out, uint64_t n, int64_t* n_samples);

/* Current distributions f = w + g as FP64 [Q][NZ][NY][NX]; synchronizes.
 * Uses the inactive buffer as staging. n = Q*NX*NY*NZ. */
int stglbm_get_f(stglbm_t h, double* h_out, uint64_t n);
/* f = w + g for the planes x0 <= x < x1 only, FP64 [Q][NZ][NY][x1-x0];
 * synchronizes; staged through the inactive buffer in pieces like get_f.
 * n = Q*NZ*NY*(x1-x0). */
int stglbm_get_f_planes(stglbm_t h, int32_t x0, int32_t x1, double* h_out, uint64_t n);
/* Device address and size in bytes of the current distributions g (store
 * type, device layout [NZ][Q][NY][NX]); valid until the next step or
 * restore. */
int stglbm_state_view(stglbm_t h, void** d_g, uint64_t* bytes);
/* Replace the distributions by f (rounded to the store type). Synchronizes. */
int stglbm_set_f(stglbm_t h, const double* h_in, uint64_t n);

/* Replace the distributions by the equilibrium f_eq(rho = 1, u) of eq.
 * local_eq, from a host velocity field u [3][NZ][NY][NX] (lattice units,
 * FP64; component-major), computed in FP64 and rounded to the store type.
 * Used to start a run from a velocity profile (e.g. the periodic reference
 * channel).  n must be 3*NX*NY*NZ.  Synchronizes. */
int stglbm_set_equilibrium(stglbm_t h, const double* h_u, uint64_t n);

/* stglbm_set_equilibrium with a physical velocity field (m/s), converted on
 * the device to lattice units by u c_t / c_x (eq. u_transfer) in FP64 before
 * f_eq is formed.  E_INVAL for non-positive c_x, c_t or a wrong n. */
int stglbm_set_equilibrium_physical(stglbm_t h, const double* h_u, uint64_t n, double c_x, double c_t);

/* Velocity probes (adaptation diagnostics: time series at chosen cells).
 * After every following step the velocity the collision used at each of the
 * n cells (x, y, z) = h_xyz[3k..3k+2] (host array, copied) is written, in
 * FP32 lattice units, to row r of the caller's device buffer d_series
 * [capacity][n][3], r = 0, 1, ... until capacity rows are written; the
 * velocity is recovered from the post-collision state as
 * (sum_i c_i f_i - F/2) / sum_i f_i.  The buffer must stay valid while
 * probes are set.  n = 0 turns probes off.  Asynchronous (one small kernel
 * per step on the handle's stream).  Errors: n outside 0..64, a cell outside
 * the lattice, null pointers or capacity < 1 give STGLBM_E_INVAL. */
#define STGLBM_MAX_PROBES 64
int stglbm_set_probes(stglbm_t h, int32_t n, const int32_t* h_xyz, float* d_series, int64_t capacity);
/* Number of probe rows written so far (enqueued; synchronize before reading). */
int stglbm_probe_rows(stglbm_t h, int64_t* rows);

/* Mode table [N][8]: k^n, d^n (3), sigma^n (3), phi^n (FP64). Synchronizes. */
int stglbm_get_modes(stglbm_t h, double* h_out, uint64_t n);
/* Per-row inlet table [NY][STGLBM_ROW_FIELDS] FP64. Synchronizes. */
#define STGLBM_ROW_FIELDS 18   /* U(3) k omega R(6) a11 a21 a22 a31 a32 a33 l_e */
int stglbm_get_inlet_rows(stglbm_t h, double* h_out, uint64_t n);
/* Inlet scalars [8]: L_e, k_min, k_max, alpha, k_cut, clamps, U_b, n_modes. */
int stglbm_get_inlet_scalars(stglbm_t h, double* h_out, uint64_t n);
/* sqrt(q^n) per row [NY][N] FP64. Synchronizes. */
int stglbm_get_sqrtq(stglbm_t h, double* h_out, uint64_t n);

/* Completed steps. */
int stglbm_get_step(stglbm_t h, int64_t* t);

/* Switch the handle to another caller-owned stream (waits for the old one
 * first). */
int stglbm_set_stream(stglbm_t h, void* hip_stream);

/* Wait for the stream and report a device-side instability. */
int stglbm_sync(stglbm_t h);

/* Checkpoint: step counter, sampling state, distributions and statistics.
 * Restoring needs a handle with the same descriptor and the same inlet input
 * (checked by a hash); a restored run continues bit for bit. */
int stglbm_checkpoint_size(stglbm_t h, uint64_t* bytes);
int stglbm_checkpoint(stglbm_t h, void* h_buf, uint64_t n);
int stglbm_restore(stglbm_t h, const void* h_buf, uint64_t n);

/* Timing of the fused step kernel and the STG kernel with HIP events on the
 * handle's stream.  enable = 0: off; enable = k >= 1: every STG launch and
 * every k-th step-kernel launch (the first after this call, then one in k),
 * so that the events' own cost (a few us per recorded launch) stays off most
 * steps.  out = {timed step-kernel ms total, timed step launches, STG-kernel
 * ms total, inlet planes generated by STG launches, STG launches[, planes
 * made by the trailing blocks of step launches (their time is part of the
 * step kernel's)]}, all counted while profiling is on; reading synchronizes
 * and clears.  n >= 5 (6 for the last value).  E_INVAL if enable < 0. */
int stglbm_profile(stglbm_t h, int32_t enable);
int stglbm_profile_read(stglbm_t h, double* out, uint64_t n);

/* Plain device copy of `bytes` (multiple of 16) on a stream: the bandwidth
 * calibration kernel for counter and roofline measurements. */
int stglbm_copy_probe(const void* d_src, void* d_dst, uint64_t bytes, void* hip_stream);

/* HBM bandwidth probes on a stream (measurement of the ceiling the step
 * kernel is compared with): mode 0 the plain copy of stglbm_copy_probe; 1 a
 * copy with four 16-byte loads in flight per lane and non-temporal stores;
 * 2 a read-only sweep of d_src (d_dst may be null; if not, its first 16
 * bytes receive the XOR of all words only when that equals one fixed 128-bit
 * constant); 3 a write-only fill of d_dst (d_src may be null).  bytes is a
 * multiple of 16.  E_INVAL for another mode or a missing buffer. */
int stglbm_bandwidth_probe(const void* d_src, void* d_dst, uint64_t bytes, int32_t mode, void* hip_stream);

/* Free the host handle (the workspace stays the caller's). */
int stglbm_destroy(stglbm_t h);

/* Last error message of a handle (or of the library if h is NULL). */
const char* stglbm_last_error(stglbm_t h);

#ifdef __cplusplus
}
#endif

#endif /* STGLBM_H */
