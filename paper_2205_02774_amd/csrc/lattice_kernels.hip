// Lattice kernels of libstglbm: the D3Q19 regularized stream-collide pass
// (the method's configuration, with 1, 2 or 4 cells per lane) and the
// helpers every configuration shares: fill, copy, sponge factors, export and
// import of f, the equilibrium start state and the velocity probes.  The
// stream-collide kernel itself is in lattice_step.h; the velocity-set and
// operator variants are instantiated in lattice_variants.hip, and the FP32
// statistics kernel of the channel steps in lattice_f32.hip.
//
// Mapping: a wave owns 64 consecutive x cells of one (y, z) row (times the
// cells per lane), so each population load and store of a wave is one
// contiguous segment.  A block is up to 8 waves at the same (x tile group, y)
// stepping through a chunk of z rows, so the per-cell statistics reduce over
// z in registers and then across the block's z waves in LDS before a single
// FP64 read-modify-write per (x, y) bin and block: fixed order, no atomics.
#include <type_traits>

#include "lattice_step.h"

namespace stglbm {
namespace {

__global__ void fill_zero_kernel(uint4* p, unsigned long long n16) {
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void stats_sum_kernel(const double* d, int nd, const float* f, int nf, long long n, double* out,
                                 bool add) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    double v = add ? out[e] : 0.0;
    for (int k = 0; k < nd; ++k) v += d[k * n + e];
    for (int k = 0; k < nf; ++k) v += static_cast<double>(f[k * n + e]);
    out[e] = v;
  }
}

// The fold of up to K window slots: every slot's value is loaded before the
// first add (the generic loop above waits for one load per slot in turn), then
// added to the FP64 total in slot order.
template <int K>
__global__ void stats_fold_kernel(const float* __restrict__ f, int nf, long long n, double* __restrict__ out) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    float x[K];
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] = k < nf ? f[k * n + e] : 0.0f;
    double v = out[e];
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < nf) v += static_cast<double>(x[k]);
    out[e] = v;
  }
}

__global__ void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, unsigned long long n16) {
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
}

// Bandwidth probes: U independent 16-byte loads in flight per lane before
// the stores (non-temporal), a read-only sweep (the XOR of what it read is
// stored only if it equals a value no buffer here holds), a write-only fill.
using U4 = unsigned __attribute__((ext_vector_type(4)));

template <int U>
__global__ void copy_wide_kernel(const U4* __restrict__ src, U4* __restrict__ dst, unsigned long long n16) {
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n16; i += U * stride) {
    U4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], &dst[i + u * stride]);
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

template <int U>
__global__ void read_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, unsigned long long n16) {
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
  uint4 acc = make_uint4(0u, 0u, 0u, 0u);
  for (; i + (U - 1) * stride < n16; i += U * stride) {
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc.x ^= v[u].x; acc.y ^= v[u].y; acc.z ^= v[u].z; acc.w ^= v[u].w;
    }
  }
  for (; i < n16; i += stride) {
    const uint4 v = src[i];
    acc.x ^= v.x; acc.y ^= v.y; acc.z ^= v.z; acc.w ^= v.w;
  }
  if (dst && acc.x == 0x9e3779b9u && acc.y == 0x7f4a7c15u && acc.z == 0xf39cc060u && acc.w == 0x5cedc834u) dst[0] = acc;
}

__global__ void write_kernel(U4* __restrict__ dst, unsigned long long n16) {
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  const U4 one = {1u, 1u, 1u, 1u};
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    __builtin_nontemporal_store(one, &dst[i]);
}

// Sponge (eq. sponge_visco): nu_sponge = nu_eff (1 + K s^p), s = (x - x_s)/(x_e - x_s),
// x_e = NX - 1, x_s = x_e - L_s; stored as the multiplier of tau - 1/2.
__global__ void sponge_kernel(float* sponge, int nx, int cells, double K, double pw) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nx) return;
  double fac = 1.0;
  if (cells > 0) {
    const int x_end = nx - 1, x_start = x_end - cells;
    if (x >= x_start) {
      const double s = static_cast<double>(x - x_start) / static_cast<double>(x_end - x_start);
      fac = K * pow(s, pw) + 1.0;
    }
  }
  sponge[x] = static_cast<float>(fac);
}

// Public element e of [Q][NZ][NY][NX] -> stored element of [NZ][Q][NY][NX].
template <int QN>
__device__ __forceinline__ long long stored_index(long long e, int nz, long long plane2d, int* pop) {
  const long long plane = static_cast<long long>(nz) * plane2d;
  const int i = static_cast<int>(e / plane);
  const long long r = e - i * plane;              // z * plane2d + (y, x)
  const long long z = r / plane2d;
  *pop = i;
  return (z * QN + i) * plane2d + (r - z * plane2d);
}

template <class Codec, int QN>
__global__ void export_f_kernel(const typename Codec::storage* g, long long offset, long long count, int nz,
                                long long plane2d, double* out) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride) {
    int i;
    const long long at = stored_index<QN>(offset + k, nz, plane2d, &i);
    out[k] = weight_d<QN>(i) + static_cast<double>(Codec::decode(g[at]));
  }
}

template <class Codec, int QN>
__global__ void export_planes_kernel(const typename Codec::storage* g, int nx, int ny, int nz, int x0, int w,
                                     long long offset, long long count, double* out) {
  const long long plane2d = (long long)nx * ny;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride) {
    const long long e = offset + k;               // element of [Q][NZ][NY][w]
    const int xx = static_cast<int>(e % w);
    const long long r = e / w;                    // (i, z, y)
    const int i = static_cast<int>(r / ((long long)nz * ny));
    const long long zy = r % ((long long)nz * ny);
    const long long z = zy / ny, y = zy % ny;
    out[k] = weight_d<QN>(i) + static_cast<double>(Codec::decode(g[(z * QN + i) * plane2d + y * nx + x0 + xx]));
  }
}

template <class Codec, int QN>
__global__ void import_f_kernel(const double* f, long long offset, long long count, int nz, long long plane2d,
                                typename Codec::storage* g) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride) {
    int i;
    const long long at = stored_index<QN>(offset + k, nz, plane2d, &i);
    g[at] = Codec::encode(static_cast<float>(f[k] - weight_d<QN>(i)));
  }
}

// f = f_eq(rho = 1, u) (eq. local_eq) from a velocity field u[3][NZ][NY][NX]
// in lattice units, computed in FP64 and rounded once to the store type.
template <class Codec, int QN>
__global__ void equilibrium_kernel(const double* u, double scale, int nx, int ny, int nz,
                                   typename Codec::storage* g) {
  const long long plane2d = (long long)nx * ny;
  const long long cells = plane2d * nz;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += stride) {
    const double ux = scale * u[c], uy = scale * u[cells + c], uz = scale * u[2 * cells + c];
    const double uu = ux * ux + uy * uy + uz * uz;
    const long long z = c / plane2d, yx = c - z * plane2d;
    for (int i = 0; i < QN; ++i) {
      const double cu = vcx<QN>(i) * ux + vcy<QN>(i) * uy + vcz<QN>(i) * uz;
      g[(z * QN + i) * plane2d + yx] = Codec::encode(static_cast<float>(weight_d<QN>(i) * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu)));
    }
  }
}

// Velocity of the collision at the probe cells, recovered from the
// post-collision state: collision keeps rho and returns sum c f = rho u + F/2
// (regularized operator with J_neq = -F/2 plus the Guo source).  FP64 sums.
template <class Codec, int QN>
__global__ void probe_kernel(ProbeParams p) {
  const int k = threadIdx.x;
  if (k >= p.n) return;
  const auto* g = static_cast<const typename Codec::storage*>(p.g);
  const long long base = (long long)p.xyz[k][2] * QN * p.plane2d + (long long)p.xyz[k][1] * p.nx + p.xyz[k][0];
  double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for (int i = 0; i < QN; ++i) {
    const double f = weight_d<QN>(i) + static_cast<double>(Codec::decode(g[base + i * p.plane2d]));
    rho += f;
    jx += vcx<QN>(i) * f;
    jy += vcy<QN>(i) * f;
    jz += vcz<QN>(i) * f;
  }
  p.out[3 * k + 0] = static_cast<float>((jx - 0.5 * p.fx) / rho);
  p.out[3 * k + 1] = static_cast<float>((jy - 0.5 * p.fy) / rho);
  p.out[3 * k + 2] = static_cast<float>((jz - 0.5 * p.fz) / rho);
}

int grid_for(unsigned long long n, int block) {
  unsigned long long b = (n + block - 1) / block;
  if (b > 65536ull * 4) b = 65536ull * 4;
  if (b < 1) b = 1;
  return static_cast<int>(b);
}

template <class Codec>
hipError_t launch_d3q19_regularized(const StepParams& p, bool stats, hipStream_t s) {
  switch (p.vec) {
    case 1: return launch_step_v<Codec, 19, true, 1>(p, stats, s);
    case 2: return launch_step_v<Codec, 19, true, 2>(p, stats, s);
    case 4: return launch_step_v<Codec, 19, true, 4>(p, stats, s);
    default: return hipErrorInvalidValue;
  }
}

// Calls f(Codec{}, std::integral_constant<int, Q>{}) for the store type and velocity set.
template <class F>
hipError_t by_store_and_set(int store, int q, F&& f) {
  using I15 = std::integral_constant<int, 15>;
  using I19 = std::integral_constant<int, 19>;
  using I27 = std::integral_constant<int, 27>;
  switch (store * 100 + q) {
    case 15: return f(CodecF32{}, I15{});
    case 19: return f(CodecF32{}, I19{});
    case 27: return f(CodecF32{}, I27{});
    case 115: return f(CodecF16{}, I15{});
    case 119: return f(CodecF16{}, I19{});
    case 127: return f(CodecF16{}, I27{});
    case 215: return f(CodecBF16{}, I15{});
    case 219: return f(CodecBF16{}, I19{});
    case 227: return f(CodecBF16{}, I27{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_step(const StepParams& p, int store, bool stats, hipStream_t s) {
  if (p.wx < 1 || p.wz < 1) return hipErrorInvalidValue;
  const int store_bytes = store == 0 ? 4 : 2;
  if (p.wx * p.wz > step_max_waves(store_bytes, p.q, p.vec, stats)) return hipErrorInvalidValue;
  if (p.vec < 1 || p.nx % p.vec != 0) return hipErrorInvalidValue;
  if (p.q != 19 || p.collision != 0) return launch_step_variant(p, store, stats, s);
  switch (store) {
    case 0: return launch_d3q19_regularized<CodecF32>(p, stats, s);
    case 1: return launch_d3q19_regularized<CodecF16>(p, stats, s);
    case 2: return launch_d3q19_regularized<CodecBF16>(p, stats, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stats_sum(const double* d, int nd, const float* f, int nf, long long n, double* out, bool add,
                            hipStream_t s) {
  const int grid = grid_for(static_cast<unsigned long long>(n), 256);
  if (nd == 0 && add && nf >= 1 && nf <= 32) {
    // the window fold: all slots' loads in flight at once
    if (nf <= 16) stats_fold_kernel<16><<<grid, 256, 0, s>>>(f, nf, n, out);
    else stats_fold_kernel<32><<<grid, 256, 0, s>>>(f, nf, n, out);
    return hipGetLastError();
  }
  stats_sum_kernel<<<grid, 256, 0, s>>>(d, nd, f, nf, n, out, add);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* ptr, unsigned long long bytes, hipStream_t s) {
  if (bytes % 16) return hipErrorInvalidValue;
  const unsigned long long n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  fill_zero_kernel<<<grid_for(n16, 256), 256, 0, s>>>(static_cast<uint4*>(ptr), n16);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, unsigned long long bytes, hipStream_t s) {
  if (bytes % 16) return hipErrorInvalidValue;
  const unsigned long long n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  copy_kernel<<<grid_for(n16, 256), 256, 0, s>>>(static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
  return hipGetLastError();
}

hipError_t launch_bandwidth_probe(const void* src, void* dst, unsigned long long bytes, int mode, hipStream_t s) {
  if (bytes % 16 || mode < 0 || mode > 3) return hipErrorInvalidValue;
  const unsigned long long n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  // one pass over the data: 4 elements per lane for modes 1 and 2, one for 0 and 3
  // (grids that loop several times over a resident set of blocks streamed slower)
  const auto* in = static_cast<const uint4*>(src);
  auto* out = static_cast<uint4*>(dst);
  const int g4 = grid_for((n16 + 3) / 4, 256);
  switch (mode) {
    case 0: copy_kernel<<<grid_for(n16, 256), 256, 0, s>>>(in, out, n16); break;
    case 1: copy_wide_kernel<4><<<g4, 256, 0, s>>>(reinterpret_cast<const U4*>(in), reinterpret_cast<U4*>(out), n16); break;
    case 2: read_kernel<4><<<g4, 256, 0, s>>>(in, out, n16); break;
    default: write_kernel<<<grid_for(n16, 256), 256, 0, s>>>(reinterpret_cast<U4*>(out), n16); break;
  }
  return hipGetLastError();
}

hipError_t launch_sponge(float* sponge, int nx, int cells, double K, double pw, hipStream_t s) {
  sponge_kernel<<<(nx + 255) / 256, 256, 0, s>>>(sponge, nx, cells, K, pw);
  return hipGetLastError();
}

hipError_t launch_export_f(const void* g, int store, int q, long long offset, long long count, int nz,
                           long long plane2d, double* out, hipStream_t s) {
  const int grid = grid_for(static_cast<unsigned long long>(count), 256);
  return by_store_and_set(store, q, [&](auto codec, auto qn) {
    using C = decltype(codec);
    export_f_kernel<C, decltype(qn)::value><<<grid, 256, 0, s>>>(static_cast<const typename C::storage*>(g), offset,
                                                                  count, nz, plane2d, out);
    return hipGetLastError();
  });
}

hipError_t launch_export_planes(const void* g, int store, int q, int nx, int ny, int nz, int x0, int x1,
                                long long offset, long long count, double* out, hipStream_t s) {
  const int w = x1 - x0;
  const int grid = grid_for(static_cast<unsigned long long>(count), 256);
  return by_store_and_set(store, q, [&](auto codec, auto qn) {
    using C = decltype(codec);
    export_planes_kernel<C, decltype(qn)::value><<<grid, 256, 0, s>>>(static_cast<const typename C::storage*>(g),
                                                                       nx, ny, nz, x0, w, offset, count, out);
    return hipGetLastError();
  });
}

hipError_t launch_import_f(const double* f, int store, int q, long long offset, long long count, int nz,
                           long long plane2d, void* g, hipStream_t s) {
  const int grid = grid_for(static_cast<unsigned long long>(count), 256);
  return by_store_and_set(store, q, [&](auto codec, auto qn) {
    using C = decltype(codec);
    import_f_kernel<C, decltype(qn)::value><<<grid, 256, 0, s>>>(f, offset, count, nz, plane2d,
                                                                  static_cast<typename C::storage*>(g));
    return hipGetLastError();
  });
}

hipError_t launch_equilibrium(const double* u, double scale, int store, int q, int nx, int ny, int nz, void* g,
                              hipStream_t s) {
  const int grid = grid_for(static_cast<unsigned long long>(nx) * ny * nz, 256);
  return by_store_and_set(store, q, [&](auto codec, auto qn) {
    using C = decltype(codec);
    equilibrium_kernel<C, decltype(qn)::value><<<grid, 256, 0, s>>>(u, scale, nx, ny, nz,
                                                                     static_cast<typename C::storage*>(g));
    return hipGetLastError();
  });
}

hipError_t launch_probes(const ProbeParams& p, int store, hipStream_t s) {
  if (p.n < 1 || p.n > kMaxProbes) return hipErrorInvalidValue;
  return by_store_and_set(store, p.q, [&](auto codec, auto qn) {
    probe_kernel<decltype(codec), decltype(qn)::value><<<1, 64, 0, s>>>(p);
    return hipGetLastError();
  });
}

}  // namespace stglbm
