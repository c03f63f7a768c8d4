// Inlet kernels of libstglbm: the one-off FP64 precompute of the synthetic
// turbulence generator and the per-step inlet velocity plane.
//
// Precompute (Algorithm 1, LBM steps 1-4), FP64: linear interpolation of the
// RANS fields to the lattice rows y_j = (j + 1/2) c_x (wall points carry
// U = k = R = 0 and the nearest omega), the Cholesky factor of R (eq.
// cholesky), l_t = sqrt(k)/(C_mu omega), l_e = min(2 d_w, C_l l_t), the
// cut-off l_cut (eq. lcut) on the uniform lattice, k_min = pi / max l_e,
// k_max = 1.5 max 2 pi / l_cut, the wavenumbers k^n = k_min (1 + alpha)^(n-1),
// the modified von Karman weights q^n (eq. qn; spectrum form of Shur et al.),
// the random directions, normals and phases (eq. dn) drawn from SplitMix64,
// and the spanwise phasor table exp(i k^n d^n_z z).
//
// Plane (steps 5-8): the phase k^n d^n . x' + phi^n of eq. psu splits into a
// row part k^n d^n_y y_j + phi^n + 2 pi d^n_x (x_in - U_b t)/L_e and a spanwise
// part k^n d^n_z z held as an FP32 phasor.  The row part's exponential is the
// product, in FP64, of a stored time-independent phasor (row, mode) and the
// time factor (mode, step), rounded once to FP32.  Their product gives cos of the full phase without a large-argument
// FP32 cosine.  A block owns 1 to 8 rows and 64 spanwise nodes of one plane
// (one launch makes the planes of up to 16 steps); its 8 waves split the
// modes, the row phasors and sigma^n are staged in LDS per chunk of modes,
// and the waves' partial sums meet in LDS.
#include <cstdlib>

#include "stglbm_internal.h"
#include "stg_block.h"

namespace stglbm {
namespace {

constexpr double kPi = 3.14159265358979323846;

// SplitMix64 (Steele, Lea & Flood 2014): output m of the stream seeded with s
// is mix(s + m * 0x9E3779B97F4A7C15); uniform double = (output >> 11) 2^-53.
__device__ __forceinline__ double splitmix_uniform(unsigned long long seed, unsigned long long m) {
  unsigned long long z = seed + m * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return static_cast<double>(z >> 11) * 0x1.0p-53;
}

__device__ double interp_field(const double* yv, const double* v, int stride, int n, double y2,
                               double yj, double wall_lo, double wall_hi) {
  // augmented grid: 0, yv[0..n-1], 2 delta with values wall_lo, v[..], wall_hi
  if (yj <= yv[0]) {
    const double t = yj / yv[0];
    return wall_lo + t * (v[0] - wall_lo);
  }
  if (yj >= yv[n - 1]) {
    const double t = (yj - yv[n - 1]) / (y2 - yv[n - 1]);
    return v[(n - 1) * stride] + t * (wall_hi - v[(n - 1) * stride]);
  }
  int lo = 0, hi = n - 1;  // yv[lo] <= yj < yv[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (yv[mid] <= yj) lo = mid; else hi = mid;
  }
  const double t = (yj - yv[lo]) / (yv[hi] - yv[lo]);
  return v[lo * stride] + t * (v[hi * stride] - v[lo * stride]);
}

__device__ __forceinline__ double cutoff_length(double dx, double dy, double dz, double dw) {
  const double dmax = fmax(dx, fmax(dy, dz));
  return 2.0 * fmin(fmax(fmax(dx, dy), 0.3 * dmax) + 0.1 * dw, dmax);
}

// Rows, length scales, wavenumber range and the mode draw; one block.
__global__ __launch_bounds__(256) void inlet_rows_kernel(SetupParams p) {
  const int tid = threadIdx.x;
  const int n = p.n_rans;
  const double* yv = p.rans;
  const double* U3 = p.rans + n;
  const double* kk = p.rans + 4 * n;
  const double* om = p.rans + 5 * n;
  const double* R6 = p.rans + 6 * n;
  const double y2 = 2.0 * p.delta;
  __shared__ double red[256];
  __shared__ int clamp_count;
  if (tid == 0) clamp_count = 0;
  __syncthreads();

  double le_max = 0.0;
  double kcut_max = 0.0;
  for (int j = tid; j < p.ny; j += blockDim.x) {
    const double yj = (j + 0.5) * p.c_x;
    const double dw = fmin(yj, y2 - yj);
    double* row = p.rows + (long long)j * kRowFields;
    for (int c = 0; c < 3; ++c) row[c] = interp_field(yv, U3 + c, 3, n, y2, yj, 0.0, 0.0);
    const double k = interp_field(yv, kk, 1, n, y2, yj, 0.0, 0.0);
    const double w = interp_field(yv, om, 1, n, y2, yj, om[0], om[n - 1]);
    double R[6];
    for (int c = 0; c < 6; ++c) R[c] = interp_field(yv, R6 + c, 6, n, y2, yj, 0.0, 0.0);
    row[3] = k;
    row[4] = w;
    for (int c = 0; c < 6; ++c) row[5 + c] = R[c];
    // Cholesky a a^T = R; R = (R11, R22, R33, R12, R13, R23)
    int clamps = 0;
    double r = R[0];
    if (r < 0.0) { ++clamps; r = 0.0; }
    const double a11 = sqrt(r);
    const double a21 = a11 > 0.0 ? R[3] / a11 : 0.0;
    const double a31 = a11 > 0.0 ? R[4] / a11 : 0.0;
    r = R[1] - a21 * a21;
    if (r < 0.0) { ++clamps; r = 0.0; }
    const double a22 = sqrt(r);
    const double a32 = a22 > 0.0 ? (R[5] - a21 * a31) / a22 : 0.0;
    r = R[2] - a31 * a31 - a32 * a32;
    if (r < 0.0) { ++clamps; r = 0.0; }
    const double a33 = sqrt(r);
    row[11] = a11; row[12] = a21; row[13] = a22; row[14] = a31; row[15] = a32; row[16] = a33;
    if (clamps) atomicAdd(&clamp_count, clamps);
    const double lt = sqrt(k) / (p.C_mu * w);
    const double le = fmin(2.0 * dw, p.C_l * lt);
    row[17] = le;
    le_max = fmax(le_max, le);
    kcut_max = fmax(kcut_max, 2.0 * kPi / cutoff_length(p.c_x, p.c_x, p.c_x, dw));
  }
  red[tid] = le_max;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  const double L_e = red[0];
  __syncthreads();
  red[tid] = kcut_max;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  const double k_min = kPi / L_e;
  const double k_max = 1.5 * red[0];
  double alpha = p.alpha;
  if (alpha <= 0.0) alpha = (p.n_modes > 1) ? pow(k_max / k_min, 1.0 / (p.n_modes - 1)) - 1.0 : 0.0;
  if (tid == 0) {
    p.scalars[0] = L_e;
    p.scalars[1] = k_min;
    p.scalars[2] = k_max;
    p.scalars[3] = alpha;
    p.scalars[4] = red[0];
    p.scalars[5] = clamp_count;
    p.scalars[6] = p.U_b;
    p.scalars[7] = p.n_modes;
    *p.clamps = clamp_count;
  }
  for (int m = tid; m < p.n_modes; m += blockDim.x) {
    const unsigned long long base = 4ull * m;
    const double Phi = 2.0 * kPi * splitmix_uniform(p.seed, base + 1);
    const double Theta = acos(1.0 - 2.0 * splitmix_uniform(p.seed, base + 2));
    const double eta = 2.0 * kPi * splitmix_uniform(p.seed, base + 3);
    const double phi = 2.0 * kPi * splitmix_uniform(p.seed, base + 4);
    double sP, cP, sT, cT, sE, cE;
    sincos(Phi, &sP, &cP);
    sincos(Theta, &sT, &cT);
    sincos(eta, &sE, &cE);
    double* md = p.modes + (long long)m * kModeFields;
    md[0] = k_min * pow(1.0 + alpha, static_cast<double>(m));
    md[1] = sT * cP;
    md[2] = sT * sP;
    md[3] = cT;
    md[4] = cP * cT * cE - sP * sE;
    md[5] = sP * cT * cE + cP * sE;
    md[6] = -sT * cE;
    md[7] = phi;
  }
}

// Modified von Karman weights per row (eq. qn): one block per row.
__global__ __launch_bounds__(256) void inlet_spectrum_kernel(SetupParams p) {
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  const double* row = p.rows + (long long)j * kRowFields;
  const double k = row[3], w = row[4], le = row[17];
  const double yj = (j + 0.5) * p.c_x;
  const double dw = fmin(yj, 2.0 * p.delta - yj);
  const double eps = p.C_mu * k * w;
  const double eta = pow(p.nu_phys * p.nu_phys * p.nu_phys / eps, 0.25);
  const double k_eta = 2.0 * kPi / eta;
  const double k_e = 2.0 * kPi / le;
  const double k_cut = 2.0 * kPi / cutoff_length(p.c_x, p.c_x, p.c_x, dw);
  const double alpha = p.scalars[3];
  double* q = p.sqrtq + (long long)j * p.n_modes;
  __shared__ double red[256];
  double sum = 0.0;
  for (int m = tid; m < p.n_modes; m += blockDim.x) {
    const double kn = p.modes[(long long)m * kModeFields];
    const double r = kn / k_e;
    const double f_eta = exp(-(12.0 * kn / k_eta) * (12.0 * kn / k_eta));
    const double c = 4.0 * fmax(kn - 0.9 * k_cut, 0.0) / k_cut;
    const double f_cut = exp(-c * c * c);
    const double E = (r * r * r * r) / pow(1.0 + 2.4 * r * r, 17.0 / 6.0) * f_eta * f_cut;
    const double e = E * alpha * kn;
    q[m] = e;
    sum += e;
  }
  red[tid] = sum;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double total = red[0];
  for (int m = tid; m < p.n_modes; m += blockDim.x) q[m] = sqrt(q[m] / total);
}

// Row phasors sqrt 6 sqrt(q^n) exp(i (k^n d^n_y y_j + phi^n)), y_j = (j + 1/2) c_x:
// the part of the plane's phase that does not change with time, FP64.
__global__ void inlet_rowphase_kernel(SetupParams p) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)p.n_modes * p.ny) return;
  const int j = static_cast<int>(e / p.n_modes);
  const int m = static_cast<int>(e % p.n_modes);
  const double* md = p.modes + (long long)m * kModeFields;
  const double sqrt6 = 2.449489742783178098;
  double s, c;
  sincos(md[0] * md[2] * ((j + 0.5) * p.c_x) + md[7], &s, &c);
  const double a = sqrt6 * p.sqrtq[e];
  p.arow[(long long)m * p.ny + j] = make_double2(a * c, a * s);   // [mode][row]
}

// Spanwise phasors exp(i k^n d^n_z z_k), z_k = k c_x, FP64 -> FP32.
__global__ void inlet_zphase_kernel(SetupParams p) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)p.n_modes * p.nz) return;
  const int m = static_cast<int>(e / p.nz);
  const int z = static_cast<int>(e % p.nz);
  const double* md = p.modes + (long long)m * kModeFields;
  double s, c;
  sincos(md[0] * md[3] * (z * p.c_x), &s, &c);
  p.bz[e] = make_float2(static_cast<float>(c), static_cast<float>(s));
  if (z == 0)
    p.sig[m] = make_float4(static_cast<float>(md[4]), static_cast<float>(md[5]), static_cast<float>(md[6]), 0.0f);
}

// Row phasors of n_planes consecutive steps into their table slots (grid y =
// plane): P[slot][m][j] = a[m][j] exp(i 2 pi d_x (x_in - U_b t) / L_e), the
// FP64 product rounded once to FP32; rows past NY (up to ptab_rows) are zero.
// A block takes kTimePhaseModes modes: their time factors (one FP64 sincos
// each) in LDS, then the rows of each mode, consecutive threads on
// consecutive rows, each thread's loads issued before its first product.
constexpr int kTimePhaseModes = 8;

__global__ __launch_bounds__(256) void stg_time_phase_kernel(StgParams p) {
  constexpr int kPer = 4;
  __shared__ double2 G[kTimePhaseModes];
  const int b = blockIdx.y;
  const int m0 = blockIdx.x * kTimePhaseModes;
  const int cnt = min(kTimePhaseModes, p.n_modes - m0);
  if (static_cast<int>(threadIdx.x) < cnt) {
    double sn, cs;
    sincos(p.modes[(long long)(m0 + threadIdx.x) * kModeFields + 1] * p.tphase[b], &sn, &cs);
    G[threadIdx.x] = make_double2(cs, sn);
  }
  __syncthreads();
  const int rows = p.ptab_rows, total = cnt * rows;
  const double2* a = p.arow + (long long)m0 * p.ny;
  float2* out = p.ptab + ((long long)p.pslot[b] * p.n_modes + m0) * rows;
  for (int e0 = threadIdx.x; e0 < total; e0 += kPer * blockDim.x) {
    double2 av[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = e0 + k * blockDim.x;
      const int mm = e / rows, j = e - mm * rows;
      av[k] = e < total && j < p.ny ? a[(long long)mm * p.ny + j] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = e0 + k * blockDim.x;
      const int mm = e / rows, j = e - mm * rows;
      if (e < total) out[e] = j < p.ny ? stg_row_phasor(av[k], G[mm]) : make_float2(0.f, 0.f);
    }
  }
}

// Inlet planes of n_planes consecutive steps (grid z), kStgRows rows x 64
// spanwise nodes per block (stg_block.h); kStgRows is chosen so that the grid
// still has >= 2048 waves.  The inlet guard |u_x| < 0.3 c_s is applied where a
// plane is used, by the step kernel.
template <int kStgRows>
__global__ __launch_bounds__(64 * kStgWaves) void stg_plane_kernel(StgParams p) {
  __shared__ __attribute__((aligned(16))) char smem[stg_block_lds<kStgRows>()];
  stg_plane_block<kStgRows, kStgInFlight>(p, blockIdx.z, blockIdx.x, blockIdx.y, threadIdx.x, threadIdx.y, smem);
}

}  // namespace

hipError_t launch_inlet_setup(const SetupParams& p, hipStream_t s) {
  inlet_rows_kernel<<<1, 256, 0, s>>>(p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  inlet_spectrum_kernel<<<p.ny, 256, 0, s>>>(p);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long n = (long long)p.n_modes * p.nz;
  inlet_zphase_kernel<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(p);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long nr = (long long)p.n_modes * p.ny;
  inlet_rowphase_kernel<<<static_cast<unsigned>((nr + 255) / 256), 256, 0, s>>>(p);
  return hipGetLastError();
}

hipError_t launch_stg_time_phase(const StgParams& p, hipStream_t s) {
  if (p.n_planes < 1 || p.n_planes > kStgBatch || p.ptab_rows < p.ny) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>((p.n_modes + kTimePhaseModes - 1) / kTimePhaseModes),
                  static_cast<unsigned>(p.n_planes));
  stg_time_phase_kernel<<<grid, 256, 0, s>>>(p);
  return hipGetLastError();
}

hipError_t launch_stg(const StgParams& p, hipStream_t s) {
  const dim3 block(64, kStgWaves);
  const long long zb = (p.nz + 63) / 64;
  if (p.n_planes < 1 || p.n_planes > kStgBatch) return hipErrorInvalidValue;
  int rows = 8;
  while (rows > 1 && zb * ((p.ny + rows - 1) / rows) * p.n_planes * kStgWaves < 2048) rows /= 2;
  if (const char* env = std::getenv("STGLBM_STG_ROWS")) {   // tuning override: 1, 2, 4 or 8
    const int r = std::atoi(env);
    if (r == 1 || r == 2 || r == 4 || r == 8) rows = r;
  }
  const dim3 grid(static_cast<unsigned>(zb), static_cast<unsigned>((p.ny + rows - 1) / rows),
                  static_cast<unsigned>(p.n_planes));
  switch (rows) {
    case 1: stg_plane_kernel<1><<<grid, block, 0, s>>>(p); break;
    case 2: stg_plane_kernel<2><<<grid, block, 0, s>>>(p); break;
    case 4: stg_plane_kernel<4><<<grid, block, 0, s>>>(p); break;
    default: stg_plane_kernel<8><<<grid, block, 0, s>>>(p); break;
  }
  return hipGetLastError();
}

}  // namespace stglbm
