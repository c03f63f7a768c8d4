// The fused stream-collide kernel of libstglbm, generic over the velocity set
// (D3Q15, D3Q19, D3Q27) and the bulk operator (regularized or plain BGK).
//
// One launch advances every cell by one time step (Algorithm 1, step 12, with
// the boundary steps 9-11 fused in): pull streaming with halfway bounce-back at
// the y walls and spanwise wrap, the regularized rebuild of the inlet (x = 0)
// and pressure-outlet (x = NX-1) nodes, the moments (eqs. density, momentum,
// tensor), the Smagorinsky relaxation time (eqs. strain, tau_eff), the sponge
// multiplier (eq. sponge_visco), the collision with the Guo force (eqs. lbe,
// local_eq, bodyforce) and, while sampling, the FP64 flow statistics.  The
// distributions live as deviations g_i = f_i - w_i so the moments are sums of
// small numbers; arithmetic is FP32.
//
// Included by the translation units that instantiate it; everything here has
// internal linkage.
#pragma once
#include "stg_block.h"
#include "stglbm_internal.h"

#include <type_traits>

namespace stglbm {
namespace {

// Velocity sets in the library's population order: rest, then opposite
// directions as neighbours (i, i+1) for odd i.  D3Q27 is D3Q19 followed by the
// 8 corners (so D3Q19 is its first 19 entries); D3Q15 is the 6 axis
// directions followed by the corners.
__constant__ constexpr int CX27[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                                       1, -1, 1, -1, 1, -1, -1, 1};
__constant__ constexpr int CY27[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                                       1, -1, 1, -1, -1, 1, 1, -1};
__constant__ constexpr int CZ27[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                                       1, -1, -1, 1, 1, -1, 1, -1};
__constant__ constexpr int CX15[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
__constant__ constexpr int CY15[15] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
__constant__ constexpr int CZ15[15] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};

template <int QN> __device__ __forceinline__ constexpr int vcx(int i) { return QN == 15 ? CX15[i] : CX27[i]; }
template <int QN> __device__ __forceinline__ constexpr int vcy(int i) { return QN == 15 ? CY15[i] : CY27[i]; }
template <int QN> __device__ __forceinline__ constexpr int vcz(int i) { return QN == 15 ? CZ15[i] : CZ27[i]; }
__device__ __forceinline__ constexpr int vopp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Lattice weights (isotropic to fourth order with c_s^2 = 1/3).
template <int QN>
__host__ __device__ constexpr double weight_d(int i) {
  if (QN == 15) return i == 0 ? 2.0 / 9.0 : (i <= 6 ? 1.0 / 9.0 : 1.0 / 72.0);
  if (QN == 27) return i == 0 ? 8.0 / 27.0 : (i <= 6 ? 2.0 / 27.0 : (i <= 18 ? 1.0 / 54.0 : 1.0 / 216.0));
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
// w_i = weight_hi + weight_lo to ~2^-48 relative (float-float pair).
template <int QN> __host__ __device__ constexpr float weight_hi(int i) { return static_cast<float>(weight_d<QN>(i)); }
template <int QN>
__host__ __device__ constexpr float weight_lo(int i) {
  return static_cast<float>(weight_d<QN>(i) - static_cast<double>(weight_hi<QN>(i)));
}
// Adding and subtracting 12 rounds |g| < 4 to a multiple of 2^-20 (ulp of [8, 16)).
constexpr float kSplit = 12.0f;

// Storage codecs: FP32 as is; FP16 and BF16 as raw 16-bit words, rounded to
// nearest even on encode, exact on decode.
struct CodecF32 {
  using storage = float;
  static __device__ __forceinline__ float decode(float v) { return v; }
  static __device__ __forceinline__ float encode(float v) { return v; }
  static __device__ __forceinline__ float from_bits(unsigned u) { return __uint_as_float(u); }
  static __device__ __forceinline__ unsigned to_bits(float v) { return __float_as_uint(v); }
};
struct CodecF16 {
  using storage = unsigned short;
  static __device__ __forceinline__ float decode(unsigned short v) {
    return static_cast<float>(__builtin_bit_cast(_Float16, v));
  }
  static __device__ __forceinline__ unsigned short encode(float v) {
    return __builtin_bit_cast(unsigned short, static_cast<_Float16>(v));
  }
  static __device__ __forceinline__ float from_bits(unsigned u) { return decode(static_cast<unsigned short>(u)); }
  static __device__ __forceinline__ unsigned to_bits(float v) { return encode(v); }
};
struct CodecBF16 {
  using storage = unsigned short;
  static __device__ __forceinline__ float decode(unsigned short v) {
    return __uint_as_float(static_cast<unsigned int>(v) << 16);
  }
  // Round to nearest even.  gfx950 converts in one instruction
  // (v_cvt_pk_bf16_f32); on 4 M values (ties, denormals, NaNs) it matched the
  // integer form bit for bit (add 0x7fff plus the lowest kept bit, keep the
  // top 16 bits; NaNs quieted), which took six instructions per population.
  static __device__ __forceinline__ unsigned short encode(float v) {
    return __builtin_bit_cast(unsigned short, static_cast<__bf16>(v));
  }
  static __device__ __forceinline__ float from_bits(unsigned u) { return __uint_as_float(u << 16); }
  static __device__ __forceinline__ unsigned to_bits(float v) { return encode(v); }
};

// w_i * S with w_i = weight_hi + weight_lo, one rounding and no systematic bias.
template <int QN>
__device__ __forceinline__ float wmul(int i, float S) {
  return __builtin_fmaf(weight_hi<QN>(i), S, weight_lo<QN>(i) * S);
}

// w_i * S for the collision outputs: the float-float product with an FP32
// store, one rounded product with a 16-bit store (whose own rounding is 2^-11
// or coarser).
template <int QN, bool EXACT>
__device__ __forceinline__ float wmul_out(int i, float S) {
  if constexpr (EXACT) return wmul<QN>(i, S);
  else return weight_hi<QN>(i) * S;
}

// Regularized rebuild of a boundary node (eqs. f_i, f_i_neq, pi_neq,
// unknown_neq, bc_eq): SIGN is the c_x of the unknown (entering) populations.
// On the known set f_neq = g - g_eq(rho, u); unknown ones mirror their opposite;
// then g_i = g_eq_i + w_i/(2 c_s^4) Q_i : Pi_neq for every i.
template <int QN, int SIGN>
__device__ __forceinline__ void regularized_rebuild(float (&g)[QN], float drho, float ux, float uy, float uz) {
  const float rho = 1.0f + drho;
  const float uu15 = 1.5f * (ux * ux + uy * uy + uz * uz);
  float seq[QN], fneq[QN];
#pragma unroll
  for (int i = 0; i < QN; ++i) {
    const float cu = vcx<QN>(i) * ux + vcy<QN>(i) * uy + vcz<QN>(i) * uz;
    seq[i] = drho + rho * (3.0f * cu + 4.5f * cu * cu - uu15);   // g_eq_i / w_i
  }
#pragma unroll
  for (int i = 0; i < QN; ++i) fneq[i] = g[i] - wmul<QN>(i, seq[i]);
#pragma unroll
  for (int i = 0; i < QN; ++i)
    if (vcx<QN>(i) == SIGN) fneq[i] = fneq[vopp(i)];
  float pxx = 0.f, pyy = 0.f, pzz = 0.f, pxy = 0.f, pxz = 0.f, pyz = 0.f;
#pragma unroll
  for (int i = 0; i < QN; ++i) {
    const int cx = vcx<QN>(i), cy = vcy<QN>(i), cz = vcz<QN>(i);
    pxx += (cx * cx) * fneq[i];
    pyy += (cy * cy) * fneq[i];
    pzz += (cz * cz) * fneq[i];
    pxy += (cx * cy) * fneq[i];
    pxz += (cx * cz) * fneq[i];
    pyz += (cy * cz) * fneq[i];
  }
  const float tr3 = (pxx + pyy + pzz) * (1.0f / 3.0f);
#pragma unroll
  for (int i = 0; i < QN; ++i) {
    const int cx = vcx<QN>(i), cy = vcy<QN>(i), cz = vcz<QN>(i);
    const float qp = (cx * cx) * pxx + (cy * cy) * pyy + (cz * cz) * pzz +
                     2.0f * ((cx * cy) * pxy + (cx * cz) * pxz + (cy * cz) * pyz) - tr3;
    g[i] = wmul<QN>(i, seq[i] + 4.5f * qp);
  }
}

// Balanced summation tree of a[O], ..., a[O + N - 1].
template <int N, int O = 0>
__device__ __forceinline__ float tree_sum(const float* a) {
  if constexpr (N == 1) {
    return a[O];
  } else {
    constexpr int H = N / 2;
    return tree_sum<H, O>(a) + tree_sum<N - H, O + H>(a);
  }
}
// sum over pairs p of c_A(2p+1) d[p] (c_A in {-1, 0, 1})
template <int QN, int A>
__device__ __forceinline__ float pair_dot(const float* d) {
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < (QN - 1) / 2; ++q) {
    const int a = 2 * q + 1;
    const int c = A == 0 ? vcx<QN>(a) : (A == 1 ? vcy<QN>(a) : vcz<QN>(a));
    if (c > 0) s += d[q];
    else if (c < 0) s -= d[q];
  }
  return s;
}
// sum over pairs p of c_A c_B (2p+1) d[p]
template <int QN, int A, int B>
__device__ __forceinline__ float pair_dot2(const float* d) {
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < (QN - 1) / 2; ++q) {
    const int a = 2 * q + 1;
    const int ca = A == 0 ? vcx<QN>(a) : (A == 1 ? vcy<QN>(a) : vcz<QN>(a));
    const int cb = B == 0 ? vcx<QN>(a) : (B == 1 ? vcy<QN>(a) : vcz<QN>(a));
    if (ca * cb > 0) s += d[q];
    else if (ca * cb < 0) s -= d[q];
  }
  return s;
}

// Buffer resource word 3 for gfx9-family targets (raw, untyped dword access).
constexpr int kBufferWord3 = 0x00020000;

// Raw buffer access of NB bytes per lane, held as kWords 32-bit words (a
// 16-bit access uses the low half of one word).
template <int NB>
struct Raw {
  static constexpr int kWords = NB < 4 ? 1 : NB / 4;
  using W2 = unsigned __attribute__((ext_vector_type(2)));
  using W4 = unsigned __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s,
                                              unsigned (&w)[kWords]) {
    if constexpr (NB == 2) {
      w[0] = __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0);
    } else if constexpr (NB == 4) {
      w[0] = __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0);
    } else if constexpr (NB == 8) {
      const W2 t = __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0);
      w[0] = t[0];
      w[1] = t[1];
    } else {
      const W4 t = __builtin_amdgcn_raw_buffer_load_b128(r, v, s, 0);
      w[0] = t[0];
      w[1] = t[1];
      w[2] = t[2];
      w[3] = t[3];
    }
  }
  // Stores are non-temporal (aux = 2): the lines are next read one step later.
  static __device__ __forceinline__ void store(const unsigned (&w)[kWords], __amdgpu_buffer_rsrc_t r, unsigned v,
                                               unsigned s) {
    if constexpr (NB == 2) {
      __builtin_amdgcn_raw_buffer_store_b16(static_cast<unsigned short>(w[0]), r, v, s, 2);
    } else if constexpr (NB == 4) {
      __builtin_amdgcn_raw_buffer_store_b32(w[0], r, v, s, 2);
    } else if constexpr (NB == 8) {
      const W2 t = {w[0], w[1]};
      __builtin_amdgcn_raw_buffer_store_b64(t, r, v, s, 2);
    } else {
      const W4 t = {w[0], w[1], w[2], w[3]};
      __builtin_amdgcn_raw_buffer_store_b128(t, r, v, s, 2);
    }
  }
};

// Element k of a lane's vector of SB-byte elements.
template <int SB>
__device__ __forceinline__ unsigned element(const unsigned* w, int k) {
  if constexpr (SB == 4) return w[k];
  else return (w[k >> 1] >> ((k & 1) * 16)) & 0xffffu;
}

// Whole-wave lane shifts (DPP): lane l receives lane l-1 (shr) or l+1 (shl);
// the wave's first (shr) or last (shl) lane receives 0.
__device__ __forceinline__ unsigned from_previous_lane(unsigned v) {
  return __builtin_amdgcn_update_dpp(0u, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ unsigned from_next_lane(unsigned v) {
  return __builtin_amdgcn_update_dpp(0u, v, 0x130, 0xf, 0xf, false);
}

// Mapping: lane l of the wave at x tile t owns the V consecutive cells
// x0 = (64 t + l) V .. x0 + V - 1 of one (y, z) row, so each population load
// and store of a lane is one V-element vector and a wave's access is one
// contiguous 64 V-element segment.  With V = 1 (the default) a lane loads the
// source cell x - c_x itself.  With V > 1, pull streaming shifts by one cell
// along x: the element that crosses a lane boundary comes from the
// neighbouring lane by a DPP shift, and only the first and last lanes of a
// wave load it from memory.
//
// In 16-bit statistics launches without a body force, blocks past the
// lattice's (blockIdx.x >= p.nblocks) make part of the inlet plane of a later
// step (stg_block.h, kStgTailRows rows x 64 spanwise nodes each).  They are
// dispatched after every lattice block and take slots as the last round of
// lattice blocks drains.  FP32 statistics launches run one round of 16-wave
// blocks, one per compute unit: there the plane blocks would run past the
// last lattice block, so those launches leave the path out, and so do the
// other instantiations (it would raise their registers and cost occupancy).
template <bool kPath, int SB>
constexpr bool kStgTail = kPath && SB == 2;

template <class Codec, int QN, bool REG, int V, bool STATS, bool FORCE>
__global__ __launch_bounds__(64 * step_max_waves(sizeof(typename Codec::storage), QN, V, STATS)) void step_kernel(StepParams p) {
  using S = typename Codec::storage;
  constexpr int SB = static_cast<int>(sizeof(S));
  if (kStgTail<STATS && !FORCE, SB> && blockIdx.x >= p.nblocks) {
    extern __shared__ __attribute__((aligned(16))) char stg_smem[];
    const int item = blockIdx.x - p.nblocks;
    const int w = (threadIdx.x >> 6) + (blockDim.x >> 6) * threadIdx.y;
    stg_plane_block<kStgTailRows, kStgTailInFlight>(p.stg, 0, item % p.stg_zb, item / p.stg_zb, threadIdx.x & 63, w,
                                                    stg_smem);
    return;
  }
  using Vec = Raw<V * SB>;
  using One = Raw<SB>;
  constexpr int NW = Vec::kWords;
  const int lane = threadIdx.x & 63;
  // every 64 consecutive threadIdx.x form one wave: wave indices are uniform
  const int wxi = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wz = __builtin_amdgcn_readfirstlane(threadIdx.y);
  int b = blockIdx.x;
  if (p.remap) {
    // Workgroups go to the 8 XCDs in turn (blockIdx.x mod 8).  When a row
    // spans several blocks (nxg > 1), give the nxg blocks of a row to one XCD,
    // so the lines that the +-1 x shifts share stay in one L2, while
    // consecutive rows still rotate over the XCDs.
    const int xcd = b & 7, k = b >> 3;
    b = ((k / p.nxg) * 8 + xcd) * p.nxg + k % p.nxg;
  }
  const int xg = b % p.nxg;
  const int rest = b / p.nxg;
  const int y = rest % p.ny;
  const int slot = rest / p.ny;
  const int xt = xg * p.wx + wxi;
  const bool wave_live = xt < p.nxt;        // waves past the last x tile only join the reduction
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  // The store is [NZ][Q][NY][NX]: one z slice holds all Q populations.  A
  // raw buffer resource spans one slice (under 4 GiB); the scalar offset is
  // population * NY NX + row start, the per-lane offset is x.
  const unsigned pop_bytes = static_cast<unsigned>(p.plane2d) * SB;
  const unsigned slice_bytes = static_cast<unsigned>(QN) * pop_bytes;
  const long long slice = static_cast<long long>(QN) * p.plane2d;
  S* const gin = const_cast<S*>(static_cast<const S*>(p.gin));
  S* const gout = static_cast<S*>(p.gout);

  // Lanes past the end of a ragged row work on the row's last V cells and
  // store nothing; they are left out of the statistics and flags.
  const int xl = (xt * 64 + lane) * V;
  const bool active = xl < nx;
  const int x0 = active ? xl : nx - V;
  // The cells just outside the lane's vector, x0 - 1 and x0 + V: wrapped when
  // x is periodic, else clamped (they only feed the entering populations of
  // the inlet and outlet nodes, which are rebuilt).
  int xm = x0 - 1, xp = x0 + V;
  if (p.periodic_x) {
    xm = xm < 0 ? nx - 1 : xm;
    xp = xp >= nx ? 0 : xp;
  } else {
    xm = xm < 0 ? 0 : xm;
    xp = xp >= nx ? nx - 1 : xp;
  }
  const bool edge_m = lane == 0;                       // no previous lane in the wave
  const bool edge_p = lane == 63 || x0 + V >= nx;      // no next lane holding x0 + V
  const unsigned v_here = static_cast<unsigned>(x0 * SB);
  const unsigned v_m = static_cast<unsigned>(xm * SB);
  const unsigned v_p = static_cast<unsigned>(xp * SB);
  const bool inlet = !p.periodic_x && x0 == 0;         // the lane's cell 0
  const bool outlet = !p.periodic_x && x0 + V == nx;   // the lane's cell V - 1
  float sp[V];
#pragma unroll
  for (int k = 0; k < V; ++k) sp[k] = p.sponge[x0 + k];

  float acc[9][V];
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int k = 0; k < V; ++k) acc[q][k] = 0.0f;
  int bad = 0;
  int bad_inlet = 0;

  // The block's waves take wz consecutive z rows and march lw times by zstep:
  // zstep = slots * wz interleaves the blocks of one (x group, y) over z, so
  // the blocks resident at a time cover one contiguous band of z per
  // population plane; zstep = wz gives each block a contiguous z chunk.
  int z0 = slot * p.wz * (p.zstep == p.wz ? p.lw : 1) + wz;
  int trips = p.lw;
  if (STATS && p.zsched) {
    // unequal chunks, longest first: slot s takes rows zbeg[s] .. zbeg[s + 1] - 1
    const int zb = p.zbeg[slot], ze = p.zbeg[slot + 1];
    z0 = zb + wz;
    trips = (ze - zb) / p.wz;
  }
  // Statistics launches may keep the block's waves in step (a barrier per z
  // row, p.lockstep), so neighbouring waves read the cache lines they share
  // while both are in L2.  Every wave of such a block makes the same trips:
  // z - wz depends only on the block, and the waves past the last x tile or
  // past the last z row go round the loop too.
  const bool lockstep = STATS && p.lockstep;
  // Source rows depend on y only: population, row and bounce-back choice.
  const unsigned row_here = static_cast<unsigned>(y * nx) * SB;
  unsigned so[QN];
  bool wall[QN];
#pragma unroll
  for (int i = 0; i < QN; ++i) {
    const int ys = y - vcy<QN>(i);
    wall[i] = ys < 0 || ys >= ny;                       // uniform over the block
    const int pop = wall[i] ? vopp(i) : i;
    const unsigned row = wall[i] ? row_here : static_cast<unsigned>(ys * nx) * SB;
    // uniform by construction; readfirstlane keeps it in a scalar register
    // (a vector copy would make the compiler loop over lanes for the load)
    so[i] = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(pop) * pop_bytes + row);
  }
  // pull streaming: g_i(x) <- g_i(x - c_i); bounce-back g_opp(i)(x) behind a wall
  unsigned w[QN][NW];
  auto load_row = [&](int zz) {
    const int zzm = zz == 0 ? nz - 1 : zz - 1;
    const int zzp = zz == nz - 1 ? 0 : zz + 1;
    const __amdgpu_buffer_rsrc_t r3[3] = {
        __builtin_amdgcn_make_buffer_rsrc(gin + zzm * slice, (short)0, slice_bytes, kBufferWord3),
        __builtin_amdgcn_make_buffer_rsrc(gin + zz * slice, (short)0, slice_bytes, kBufferWord3),
        __builtin_amdgcn_make_buffer_rsrc(gin + zzp * slice, (short)0, slice_bytes, kBufferWord3)};
#pragma unroll
    for (int i = 0; i < QN; ++i) {
      const __amdgpu_buffer_rsrc_t r = wall[i] ? r3[1] : r3[1 - vcz<QN>(i)];
      // one cell per lane: load the source cell x - c_x directly
      const unsigned voff = (V > 1 || wall[i] || vcx<QN>(i) == 0) ? v_here : (vcx<QN>(i) > 0 ? v_m : v_p);
      Vec::load(r, voff, so[i], w[i]);
    }
  };
  // In FP32 statistics launches (several z rows per wave, one cell per lane)
  // the next row's loads are issued after this row's arithmetic and before
  // its stores, so waiting for them does not wait for the stores (the memory
  // counter is in order): 512x128x256 0.498 -> 0.481 ms.  The 16-bit launches
  // measured no gain (BF16 a loss) and keep the loads at the top of the loop.
  constexpr bool kPipe = STATS && V == 1 && SB == 4;
  if (kPipe && wave_live && z0 < nz && trips > 0) load_row(z0);
  for (int it = 0; it < ((wave_live || lockstep) ? trips : 0); ++it) {
    const int z = z0 + it * p.zstep;
    if (lockstep) {
      if (z - wz >= nz) break;
      __syncthreads();
      if (!wave_live || z >= nz) continue;
    } else if (z >= nz) {
      break;
    }
    const int zm = z == 0 ? nz - 1 : z - 1;
    const int zp = z == nz - 1 ? 0 : z + 1;
    // source slices z - c_z for c_z = +1, 0, -1, and the destination slice
    const __amdgpu_buffer_rsrc_t rin[3] = {
        __builtin_amdgcn_make_buffer_rsrc(gin + zm * slice, (short)0, slice_bytes, kBufferWord3),
        __builtin_amdgcn_make_buffer_rsrc(gin + z * slice, (short)0, slice_bytes, kBufferWord3),
        __builtin_amdgcn_make_buffer_rsrc(gin + zp * slice, (short)0, slice_bytes, kBufferWord3)};
    const __amdgpu_buffer_rsrc_t rout =
        __builtin_amdgcn_make_buffer_rsrc(gout + z * slice, (short)0, slice_bytes, kBufferWord3);
    if (!kPipe) load_row(z);
    // cross-lane elements of the x-moving populations (bounce-back ones stay put)
    unsigned ext[QN];
#pragma unroll
    for (int i = 0; i < QN; ++i) ext[i] = 0u;
    if (V > 1 && edge_m) {
#pragma unroll
      for (int i = 0; i < QN; ++i)
        if (vcx<QN>(i) > 0 && !wall[i]) {
          unsigned e[1];
          One::load(rin[1 - vcz<QN>(i)], v_m, so[i], e);
          ext[i] = e[0];
        }
    }
    if (V > 1 && edge_p) {
#pragma unroll
      for (int i = 0; i < QN; ++i)
        if (vcx<QN>(i) < 0 && !wall[i]) {
          unsigned e[1];
          One::load(rin[1 - vcz<QN>(i)], v_p, so[i], e);
          ext[i] = e[0];
        }
    }
#pragma unroll
    for (int i = 0; i < QN; ++i) {
      if (V == 1) {
        ext[i] = element<SB>(&w[i][0], 0);
      } else if (vcx<QN>(i) > 0) {
        const unsigned t = element<SB>(&w[i][0], V - 1);
        const unsigned sh = from_previous_lane(t);
        ext[i] = edge_m ? ext[i] : sh;
      } else if (vcx<QN>(i) < 0) {
        const unsigned sh = from_next_lane(element<SB>(&w[i][0], 0));
        ext[i] = edge_p ? ext[i] : sh;
      }
    }

    float ubx = 0.f, uby = 0.f, ubz = 0.f;
    if (inlet) {
      const float* u = p.ubc + 3 * (y * nz + z);
      ubx = u[0];
      uby = u[1];
      ubz = u[2];
      bad_inlet |= !(__builtin_fabsf(ubx) < p.mach_limit);   // density_bc needs |u_x| well below c_s
    }

    unsigned out[QN][NW];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      float g[QN];
#pragma unroll
      for (int i = 0; i < QN; ++i) {
        unsigned bits;
        if (vcx<QN>(i) == 0) bits = element<SB>(&w[i][0], k);
        else if (vcx<QN>(i) > 0) bits = wall[i] ? element<SB>(&w[i][0], k) : (k == 0 ? ext[i] : element<SB>(&w[i][0], k - 1));
        else bits = wall[i] ? element<SB>(&w[i][0], k) : (k == V - 1 ? ext[i] : element<SB>(&w[i][0], k + 1));
        g[i] = Codec::from_bits(bits);
      }

      if (k == 0 && inlet) {
        float g0 = 0.f, gm = 0.f;
#pragma unroll
        for (int i = 0; i < QN; ++i) {
          if (vcx<QN>(i) == 0) g0 += g[i];
          if (vcx<QN>(i) == -1) gm += g[i];
        }
        // Zou-He (eq. density_bc): rho (1 - u_x) = sum_{c_x=0} f + 2 sum_{c_x=-1} f
        const float drho = (g0 + 2.0f * gm + ubx) / (1.0f - ubx);
        regularized_rebuild<QN, 1>(g, drho, ubx, uby, ubz);
      }
      if (k == V - 1 && outlet) {
        float g0 = 0.f, gp = 0.f;
#pragma unroll
        for (int i = 0; i < QN; ++i) {
          if (vcx<QN>(i) == 0) g0 += g[i];
          if (vcx<QN>(i) == 1) gp += g[i];
        }
        // rho_out (1 + u_x) = sum_{c_x=0} f + 2 sum_{c_x=+1} f, tangential u = 0
        const float ux = (g0 + 2.0f * gp - p.rho_out_m1) * p.inv_rho_out;
        regularized_rebuild<QN, -1>(g, p.rho_out_m1, ux, 0.0f, 0.0f);
      }

      // Moments.  With an FP32 store each g is split into hi (rounded to a
      // multiple of 2^-20, so integer combinations of hi are exact in FP32
      // while |sum| < 16) and lo = g - hi (exact); opposite pairs (a, a+1)
      // give exact sums and differences.  A 16-bit store rounds g to 2^-11 or
      // 2^-8 relative every step, far above the rounding of plain FP32 sums,
      // so those launches sum directly and save about a third of the
      // arithmetic (they are bound by it, not by HBM).
      constexpr int NP = (QN - 1) / 2;
      constexpr bool kExact = SB == 4;
      float sg[NP];
      float dh, dl, jxh, jyh, jzh, jxl, jyl, jzl;
      if constexpr (kExact) {
        float h[QN], l[QN];
#pragma unroll
        for (int i = 0; i < QN; ++i) {
          h[i] = (g[i] + kSplit) - kSplit;
          l[i] = g[i] - h[i];
        }
        float sh[NP], dhh[NP], sl[NP], dll[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const int a = 2 * q + 1;
          sh[q] = h[a] + h[a + 1];
          dhh[q] = h[a] - h[a + 1];
          sl[q] = l[a] + l[a + 1];
          dll[q] = l[a] - l[a + 1];
          sg[q] = g[a] + g[a + 1];
        }
        dh = h[0] + tree_sum<NP>(sh);
        dl = l[0] + tree_sum<NP>(sl);
        // sum c g as hi + lo (each pair contributes c_a (g_a - g_opp))
        jxh = pair_dot<QN, 0>(dhh); jyh = pair_dot<QN, 1>(dhh); jzh = pair_dot<QN, 2>(dhh);
        jxl = pair_dot<QN, 0>(dll); jyl = pair_dot<QN, 1>(dll); jzl = pair_dot<QN, 2>(dll);
      } else {
        float dg[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const int a = 2 * q + 1;
          sg[q] = g[a] + g[a + 1];
          dg[q] = g[a] - g[a + 1];
        }
        dh = g[0] + tree_sum<NP>(sg);
        dl = 0.0f;
        jxh = pair_dot<QN, 0>(dg); jyh = pair_dot<QN, 1>(dg); jzh = pair_dot<QN, 2>(dg);
        jxl = jyl = jzl = 0.0f;
      }
      const float drho = dh + dl;
      const float gsum = kExact ? g[0] + tree_sum<NP>(sg) : dh;
      // sum (3 c_a c_b - delta_ab) g: 3 (pair sums weighted by c_a c_b) - delta_ab sum g
      const float hxx = 3.0f * pair_dot2<QN, 0, 0>(sg) - gsum;
      const float hyy = 3.0f * pair_dot2<QN, 1, 1>(sg) - gsum;
      const float hzz = 3.0f * pair_dot2<QN, 2, 2>(sg) - gsum;
      const float hxy = 3.0f * pair_dot2<QN, 0, 1>(sg);
      const float hxz = 3.0f * pair_dot2<QN, 0, 2>(sg);
      const float hyz = 3.0f * pair_dot2<QN, 1, 2>(sg);

      const float rho = 1.0f + drho;
      float irho = __builtin_amdgcn_rcpf(rho);
      irho = __builtin_fmaf(irho, __builtin_fmaf(-rho, irho, 1.0f), irho);   // one Newton step
      // rho u = sum c f + F/2 (eq. momentum)
      const float ux = ((jxh + jxl) + (FORCE ? 0.5f * p.fx : 0.0f)) * irho;
      const float uy = ((jyh + jyl) + (FORCE ? 0.5f * p.fy : 0.0f)) * irho;
      const float uz = ((jzh + jzl) + (FORCE ? 0.5f * p.fz : 0.0f)) * irho;
      bad |= !(fabsf(drho) < 0.5f);

      // Pi_neq = sum c c (f - f_eq) = sum (c c - c_s^2 I) g - rho u u
      const float nxx = hxx * (1.0f / 3.0f) - rho * ux * ux;
      const float nyy = hyy * (1.0f / 3.0f) - rho * uy * uy;
      const float nzz = hzz * (1.0f / 3.0f) - rho * uz * uz;
      const float nxy = hxy * (1.0f / 3.0f) - rho * ux * uy;
      const float nxz = hxz * (1.0f / 3.0f) - rho * ux * uz;
      const float nyz = hyz * (1.0f / 3.0f) - rho * uy * uz;
      const float q2 = nxx * nxx + nyy * nyy + nzz * nzz + 2.0f * (nxy * nxy + nxz * nxz + nyz * nyz);
      // tau_eff - 1/2 = (tau0 - 1/2) + X / (2 (sqrt(tau0^2 + X) + tau0)), X = 18 sqrt2 Cs^2 Q^1/2 / rho
      const float X = p.c18 * __builtin_amdgcn_sqrtf(q2) * irho;
      const float s = (p.s0 + X * __builtin_amdgcn_rcpf(2.0f * (__builtin_amdgcn_sqrtf(p.tau0_sq + X) + p.tau0))) * sp[k];
      const float itau = __builtin_amdgcn_rcpf(0.5f + s);
      const float omw = (s - 0.5f) * itau;      // 1 - 1/tau
      const float omw45 = 4.5f * omw;
      const float tr3 = (nxx + nyy + nzz) * (1.0f / 3.0f);
      const float uu15 = 1.5f * (ux * ux + uy * uy + uz * uz);
      const float omhw = FORCE ? s * itau : 0.0f;         // 1 - 1/(2 tau)
      const float uF = FORCE ? ux * p.fx + uy * p.fy + uz * p.fz : 0.0f;

      float o[QN];
      if constexpr (REG) {
        // Regularized operator.  For a pair (a, opp(a)) with velocity c:
        //   g'/w = [drho + 3 c.J] + rho (4.5 (c.u)^2 - 1.5 u.u) + (1 - 1/tau) 4.5 Q:Pi_neq (+ force terms)
        // the bracket is exact from the hi parts (big, odd in c); everything else is
        // small and split into an even part E and an odd part O.  w_i is applied as
        // w_hi S + w_lo S (one rounding, no systematic bias from rounding w_i).
        const float base_e = dl - rho * uu15;
        {
          // rest population: c = 0
          float e0 = base_e + omw45 * (-tr3);
          if (FORCE) e0 += -3.0f * omhw * uF;
          o[0] = wmul_out<QN, kExact>(0, dh + e0);
        }
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const int a = 2 * q + 1;
          const int cx = vcx<QN>(a), cy = vcy<QN>(a), cz = vcz<QN>(a);
          const float cu = cx * ux + cy * uy + cz * uz;
          const float qp = (cx * cx) * nxx + (cy * cy) * nyy + (cz * cz) * nzz +
                           2.0f * ((cx * cy) * nxy + (cx * cz) * nxz + (cy * cz) * nyz) - tr3;
          float E = __builtin_fmaf(rho * 4.5f * cu, cu, base_e) + omw45 * qp;
          const float Oh = 3.0f * (cx * jxh + cy * jyh + cz * jzh);     // exact
          float Ol = 3.0f * (cx * jxl + cy * jyl + cz * jzl);
          if (FORCE) {
            const float cF = cx * p.fx + cy * p.fy + cz * p.fz;
            E += omhw * (9.0f * cu * cF - 3.0f * uF);
            Ol += cF * (1.5f * (1.0f - omw) + 3.0f * omhw);
          }
          o[a] = wmul_out<QN, kExact>(a, (dh + Oh) + (E + Ol));
          o[a + 1] = wmul_out<QN, kExact>(a + 1, (dh - Oh) + (E - Ol));
        }
      } else {
        // Plain BGK (eq. lbe): g' = (1 - 1/tau) g + (1/tau) g_eq + Guo source, with
        // g_eq/w = drho + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u) split into even and odd parts.
        {
          float e0 = itau * (drho - rho * uu15);
          if (FORCE) e0 += -3.0f * omhw * uF;
          o[0] = __builtin_fmaf(omw, g[0], wmul_out<QN, kExact>(0, e0));
        }
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const int a = 2 * q + 1;
          const int cx = vcx<QN>(a), cy = vcy<QN>(a), cz = vcz<QN>(a);
          const float cu = cx * ux + cy * uy + cz * uz;
          float E = itau * (drho + rho * (4.5f * cu * cu) - rho * uu15);
          float O = itau * (3.0f * rho * cu);
          if (FORCE) {
            const float cF = cx * p.fx + cy * p.fy + cz * p.fz;
            E += omhw * (9.0f * cu * cF - 3.0f * uF);
            O += 3.0f * omhw * cF;
          }
          o[a] = __builtin_fmaf(omw, g[a], wmul_out<QN, kExact>(a, E + O));
          o[a + 1] = __builtin_fmaf(omw, g[a + 1], wmul_out<QN, kExact>(a + 1, E - O));
        }
      }
#pragma unroll
      for (int i = 0; i < QN; ++i) {
        const unsigned bits = Codec::to_bits(o[i]);
        if constexpr (SB == 4) out[i][k] = bits;
        else if ((k & 1) == 0) out[i][k >> 1] = bits;
        else out[i][k >> 1] |= bits << 16;
      }

      if (STATS) {
        acc[0][k] += ux;
        acc[1][k] += uy;
        acc[2][k] += uz;
        acc[3][k] += ux * ux;
        acc[4][k] += uy * uy;
        acc[5][k] += uz * uz;
        acc[6][k] += ux * uy;
        acc[7][k] += ux * uz;
        acc[8][k] += uy * uz;
      }
    }

    if (kPipe && it + 1 < trips && z + p.zstep < nz) load_row(z + p.zstep);
    if (active) {
#pragma unroll
      for (int i = 0; i < QN; ++i)
        Vec::store(out[i], rout, v_here, static_cast<unsigned>(i) * pop_bytes + row_here);
    }
  }

  // one flag write per wave
  if (__any(bad && active && wave_live)) {
    if (lane == 0) atomicOr(p.flag, kFlagDensity);
  }
  if (__any(bad_inlet)) {
    if (lane == 0) atomicOr(p.flag, kFlagInletMach);
  }

  if (STATS) {
    // per-(x, y) sums over the block's z range: registers, then the wz waves in
    // LDS.  All 9 slot values are loaded first, before the barrier: a
    // read-modify-write per quantity would make 9 dependent round trips (the
    // stores may alias the later loads as far as the compiler knows).
    // Each slot holds FP32 sums over a window of kStatsWindow sampled steps
    // (half the bytes of FP64 slots), which the host folds into FP64 totals
    // after the window's last step.
    using Acc = float;
    extern __shared__ float red[];             // [wz][9][64 wx V]
    const int tx = threadIdx.x, bx = 64 * p.wx * V;
    const bool rmw = wz == 0 && active && wave_live;
    const long long sstride = (long long)ny * nx;
    Acc* st = p.win + (long long)slot * 9 * sstride + (long long)y * nx + x0;
    const bool fresh = p.win_first;
    Acc old[9][V];
    if (rmw) {
#pragma unroll
      for (int q = 0; q < 9; ++q)
#pragma unroll
        for (int k = 0; k < V; ++k) old[q][k] = fresh ? Acc(0) : st[q * sstride + k];
    }
    if (p.wz > 1) {
#pragma unroll
      for (int q = 0; q < 9; ++q)
#pragma unroll
        for (int k = 0; k < V; ++k) red[(wz * 9 + q) * bx + tx * V + k] = acc[q][k];
      __syncthreads();
    }
    if (rmw) {
#pragma unroll
      for (int q = 0; q < 9; ++q)
#pragma unroll
        for (int k = 0; k < V; ++k) {
          float v = acc[q][k];
          for (int w = 1; w < p.wz; ++w) v += red[(w * 9 + q) * bx + tx * V + k];
          st[q * sstride + k] = old[q][k] + static_cast<Acc>(v);
        }
    }
  }
}

}  // namespace

// FP32 statistics kernels without a body force (one cell per lane) built
// with the machine scheduler set for instruction-level parallelism, in their
// own unit, lattice_f32.hip: D3Q15 regularized and D3Q19 plain BGK always;
// D3Q19 regularized (the channel's) when p.f32_ilp is set, its default being
// the copy built here with the default schedule.
template <int QN, bool REG>
constexpr bool kIlpUnit = (QN == 15 && REG) || (QN == 19 && !REG);
template <int QN, bool REG>
hipError_t launch_f32_stats(const StepParams& p, dim3 grid, dim3 block, size_t lds, hipStream_t s);

namespace {

template <class Codec, int QN, bool REG, int V>
hipError_t launch_step_v(const StepParams& p, bool stats, hipStream_t s) {
  const dim3 block(64 * p.wx, p.wz);
  // trailing plane blocks: 16-bit statistics launches without a force, kStgWaves waves per block
  if (p.stg_blocks > 0 && (!stats || p.has_force || sizeof(typename Codec::storage) != 2 || p.wx * p.wz < kStgWaves))
    return hipErrorInvalidValue;
  const dim3 grid(p.nblocks + p.stg_blocks);
  size_t lds = (stats && p.wz > 1) ? sizeof(float) * 9 * 64 * V * p.wx * p.wz : 0;
  constexpr size_t kStgLds = stg_block_lds<kStgTailRows>();
  if (p.stg_blocks > 0 && lds < kStgLds) lds = kStgLds;
  if (p.has_force) {
    if (stats) step_kernel<Codec, QN, REG, V, true, true><<<grid, block, lds, s>>>(p);
    else step_kernel<Codec, QN, REG, V, false, true><<<grid, block, lds, s>>>(p);
  } else {
    if constexpr (std::is_same_v<Codec, CodecF32> && V == 1 && kIlpUnit<QN, REG>) {
      if (stats) return launch_f32_stats<QN, REG>(p, grid, block, lds, s);
    } else {
      if constexpr (std::is_same_v<Codec, CodecF32> && V == 1 && QN == 19 && REG) {
        if (stats && p.f32_ilp) return launch_f32_stats<QN, REG>(p, grid, block, lds, s);
      }
      if (stats) step_kernel<Codec, QN, REG, V, true, false><<<grid, block, lds, s>>>(p);
    }
    if (!stats) step_kernel<Codec, QN, REG, V, false, false><<<grid, block, lds, s>>>(p);
  }
  return hipGetLastError();
}

}  // namespace
}  // namespace stglbm
