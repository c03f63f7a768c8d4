// Lattice kernels of libstglbm: the fused stream-collide pass and its helpers.
//
// One launch advances every cell by one time step (Algorithm 1, step 12, with
// the boundary steps 9-11 fused in): pull streaming with halfway bounce-back at
// the y walls and spanwise wrap, the regularized rebuild of the inlet (x = 0)
// and pressure-outlet (x = NX-1) nodes, the moments (eqs. density, momentum,
// tensor), the Smagorinsky relaxation time (eqs. strain, tau_eff), the sponge
// multiplier (eq. sponge_visco), the regularized BGK collision with the Guo
// force (eqs. lbe, local_eq, bodyforce) and, while sampling, the FP64 flow
// statistics.  The distributions live as deviations g_i = f_i - w_i so the
// moments are sums of small numbers; arithmetic is FP32.
//
// Mapping: a wave owns 64 consecutive x cells of one (y, z) row, so each of the
// 19 population loads and stores of a wave is one contiguous 256-byte (FP32)
// or 128-byte (FP16/BF16) segment.  A block is 4 waves at the same (x tile, y)
// stepping through a spanwise range, so the per-cell statistics reduce over z
// in registers and then across the 4 waves in LDS before a single FP64
// read-modify-write per (x, y) bin and block: fixed order, no atomics.  Blocks
// are renumbered so that consecutive x tiles run on the same XCD, where the
// cache lines straddled by the +-1 x shifts are shared through its L2.
#include "stglbm_internal.h"

namespace stglbm {
namespace {

// D3Q19 velocity set in the library's population order.
__constant__ constexpr int CX[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__constant__ constexpr int CY[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__constant__ constexpr int CZ[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__constant__ constexpr int OPPOSITE[kQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

__host__ __device__ constexpr double weight_d(int i) {
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
// w_i = weight_hi + weight_lo to ~2^-48 relative (float-float pair).
__host__ __device__ constexpr float weight_hi(int i) { return static_cast<float>(weight_d(i)); }
__host__ __device__ constexpr float weight_lo(int i) {
  return static_cast<float>(weight_d(i) - static_cast<double>(weight_hi(i)));
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
  static __device__ __forceinline__ unsigned short encode(float v) {
    unsigned int u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<unsigned short>((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                                             // nearest even
    return static_cast<unsigned short>(u >> 16);
  }
  static __device__ __forceinline__ float from_bits(unsigned u) { return __uint_as_float(u << 16); }
  static __device__ __forceinline__ unsigned to_bits(float v) { return encode(v); }
};

// Regularized rebuild of a boundary node (eqs. f_i, f_i_neq, pi_neq,
// unknown_neq, bc_eq): SIGN is the c_x of the unknown (entering) populations.
// On the known set f_neq = g - g_eq(rho, u); unknown ones mirror their opposite;
// then g_i = g_eq_i + w_i/(2 c_s^4) Q_i : Pi_neq for every i.
// w_i * S with w_i = weight_hi + weight_lo, one rounding and no systematic bias.
__device__ __forceinline__ float wmul(int i, float S) { return __builtin_fmaf(weight_hi(i), S, weight_lo(i) * S); }

// Regularized rebuild of a boundary node (eqs. f_i, f_i_neq, pi_neq,
// unknown_neq, bc_eq): SIGN is the c_x of the unknown (entering) populations.
// On the known set f_neq = g - g_eq(rho, u); unknown ones mirror their opposite;
// then g_i = g_eq_i + w_i/(2 c_s^4) Q_i : Pi_neq for every i.
template <int SIGN>
__device__ __forceinline__ void regularized_rebuild(float (&g)[kQ], float drho, float ux, float uy, float uz) {
  const float rho = 1.0f + drho;
  const float uu15 = 1.5f * (ux * ux + uy * uy + uz * uz);
  float seq[kQ], fneq[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const float cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
    seq[i] = drho + rho * (3.0f * cu + 4.5f * cu * cu - uu15);   // g_eq_i / w_i
  }
#pragma unroll
  for (int i = 0; i < kQ; ++i) fneq[i] = g[i] - wmul(i, seq[i]);
#pragma unroll
  for (int i = 0; i < kQ; ++i)
    if (CX[i] == SIGN) fneq[i] = fneq[OPPOSITE[i]];
  float pxx = 0.f, pyy = 0.f, pzz = 0.f, pxy = 0.f, pxz = 0.f, pyz = 0.f;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    pxx += (CX[i] * CX[i]) * fneq[i];
    pyy += (CY[i] * CY[i]) * fneq[i];
    pzz += (CZ[i] * CZ[i]) * fneq[i];
    pxy += (CX[i] * CY[i]) * fneq[i];
    pxz += (CX[i] * CZ[i]) * fneq[i];
    pyz += (CY[i] * CZ[i]) * fneq[i];
  }
  const float tr3 = (pxx + pyy + pzz) * (1.0f / 3.0f);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const float qp = (CX[i] * CX[i]) * pxx + (CY[i] * CY[i]) * pyy + (CZ[i] * CZ[i]) * pzz +
                     2.0f * ((CX[i] * CY[i]) * pxy + (CX[i] * CZ[i]) * pxz + (CY[i] * CZ[i]) * pyz) - tr3;
    g[i] = wmul(i, seq[i] + 4.5f * qp);
  }
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
// and store of a lane is one V-element vector (8 bytes by default) and a
// wave's access is one contiguous 64 V-element segment.  Pull streaming
// shifts by one cell along x: the element that crosses a lane boundary comes
// from the neighbouring lane by a DPP shift, and only the first and last
// lanes of a wave load it from memory.
template <class Codec, int V, bool STATS, bool FORCE>
__global__ __launch_bounds__(64 * kMaxWavesPerBlock) void step_kernel(StepParams p) {
  using S = typename Codec::storage;
  constexpr int SB = static_cast<int>(sizeof(S));
  using Vec = Raw<V * SB>;
  using One = Raw<SB>;
  constexpr int NW = Vec::kWords;
  const int lane = threadIdx.x & 63;
  // every 64 consecutive threadIdx.x form one wave: wave indices are uniform
  const int wxi = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wz = __builtin_amdgcn_readfirstlane(threadIdx.y);
  int b = blockIdx.x;
  if (p.remap) {
    const int per = p.nblocks >> 3;
    b = (b & 7) * per + (b >> 3);
  }
  const int xg = b % p.nxg;
  const int rest = b / p.nxg;
  const int y = rest % p.ny;
  const int slot = rest / p.ny;
  const int xt = xg * p.wx + wxi;
  const bool wave_live = xt < p.nxt;        // waves past the last x tile only join the reduction
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  // The store is [NZ][19][NY][NX]: one z slice holds all 19 populations.  A
  // raw buffer resource spans one slice (under 4 GiB); the scalar offset is
  // population * NY NX + row start, the per-lane offset is x.
  const unsigned pop_bytes = static_cast<unsigned>(p.plane2d) * SB;
  const unsigned slice_bytes = static_cast<unsigned>(kQ) * pop_bytes;
  const long long slice = static_cast<long long>(kQ) * p.plane2d;
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

  // The block's waves take wz consecutive z rows and march lw times by zstep:
  // zstep = slots * wz interleaves the blocks of one (x group, y) over z, so
  // the blocks resident at a time cover one contiguous band of z per
  // population plane; zstep = wz gives each block a contiguous z chunk.
  const int z0 = slot * p.wz * (p.zstep == p.wz ? p.lw : 1) + wz;
  for (int it = 0; it < (wave_live ? p.lw : 0); ++it) {
    const int z = z0 + it * p.zstep;
    if (z >= nz) break;
    const int zm = z == 0 ? nz - 1 : z - 1;
    const int zp = z == nz - 1 ? 0 : z + 1;
    const unsigned row_here = static_cast<unsigned>(y * nx) * SB;
    // source slices z - c_z for c_z = +1, 0, -1, and the destination slice
    const __amdgpu_buffer_rsrc_t rin[3] = {
        __builtin_amdgcn_make_buffer_rsrc(gin + zm * slice, (short)0, slice_bytes, kBufferWord3),
        __builtin_amdgcn_make_buffer_rsrc(gin + z * slice, (short)0, slice_bytes, kBufferWord3),
        __builtin_amdgcn_make_buffer_rsrc(gin + zp * slice, (short)0, slice_bytes, kBufferWord3)};
    const __amdgpu_buffer_rsrc_t rout =
        __builtin_amdgcn_make_buffer_rsrc(gout + z * slice, (short)0, slice_bytes, kBufferWord3);

    // pull streaming: g_i(x) <- g_i(x - c_i); bounce-back g_opp(i)(x) behind a wall
    unsigned w[kQ][NW];
    unsigned so[kQ];
    bool wall[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int ys = y - CY[i];
      wall[i] = ys < 0 || ys >= ny;                     // uniform over the block
      const int pop = wall[i] ? OPPOSITE[i] : i;
      const unsigned row = wall[i] ? row_here : static_cast<unsigned>(ys * nx) * SB;
      // uniform by construction; readfirstlane keeps it in a scalar register
      // (a vector copy would make the compiler loop over lanes for the load)
      so[i] = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(pop) * pop_bytes + row);
      const __amdgpu_buffer_rsrc_t r = wall[i] ? rin[1] : rin[1 - CZ[i]];
      // one cell per lane: load the source cell x - c_x directly
      const unsigned voff = (V > 1 || wall[i] || CX[i] == 0) ? v_here : (CX[i] > 0 ? v_m : v_p);
      Vec::load(r, voff, so[i], w[i]);
    }
    // cross-lane elements of the x-moving populations (bounce-back ones stay put)
    unsigned ext[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) ext[i] = 0u;
    if (V > 1 && edge_m) {
#pragma unroll
      for (int i = 0; i < kQ; ++i)
        if (CX[i] > 0 && !wall[i]) {
          unsigned e[1];
          One::load(rin[1 - CZ[i]], v_m, so[i], e);
          ext[i] = e[0];
        }
    }
    if (V > 1 && edge_p) {
#pragma unroll
      for (int i = 0; i < kQ; ++i)
        if (CX[i] < 0 && !wall[i]) {
          unsigned e[1];
          One::load(rin[1 - CZ[i]], v_p, so[i], e);
          ext[i] = e[0];
        }
    }
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      if (V == 1) {
        ext[i] = element<SB>(&w[i][0], 0);
      } else if (CX[i] > 0) {
        const unsigned t = element<SB>(&w[i][0], V - 1);
        const unsigned sh = from_previous_lane(t);
        ext[i] = edge_m ? ext[i] : sh;
      } else if (CX[i] < 0) {
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
    }

    unsigned out[kQ][NW];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      float g[kQ];
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
        unsigned bits;
        if (CX[i] == 0) bits = element<SB>(&w[i][0], k);
        else if (CX[i] > 0) bits = wall[i] ? element<SB>(&w[i][0], k) : (k == 0 ? ext[i] : element<SB>(&w[i][0], k - 1));
        else bits = wall[i] ? element<SB>(&w[i][0], k) : (k == V - 1 ? ext[i] : element<SB>(&w[i][0], k + 1));
        g[i] = Codec::from_bits(bits);
      }

      if (k == 0 && inlet) {
        float g0 = 0.f, gm = 0.f;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
          if (CX[i] == 0) g0 += g[i];
          if (CX[i] == -1) gm += g[i];
        }
        // Zou-He (eq. density_bc): rho (1 - u_x) = sum_{c_x=0} f + 2 sum_{c_x=-1} f
        const float drho = (g0 + 2.0f * gm + ubx) / (1.0f - ubx);
        regularized_rebuild<1>(g, drho, ubx, uby, ubz);
      }
      if (k == V - 1 && outlet) {
        float g0 = 0.f, gp = 0.f;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
          if (CX[i] == 0) g0 += g[i];
          if (CX[i] == 1) gp += g[i];
        }
        // rho_out (1 + u_x) = sum_{c_x=0} f + 2 sum_{c_x=+1} f, tangential u = 0
        const float ux = (g0 + 2.0f * gp - p.rho_out_m1) * p.inv_rho_out;
        regularized_rebuild<-1>(g, p.rho_out_m1, ux, 0.0f, 0.0f);
      }

      // Moments.  Each g is split into hi (rounded to a multiple of 2^-20, so
      // integer combinations of hi are exact in FP32 while |sum| < 16) and
      // lo = g - hi (exact).  Opposite pairs (a, a+1) give exact sums/differences.
      float h[kQ], l[kQ];
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
        h[i] = (g[i] + kSplit) - kSplit;
        l[i] = g[i] - h[i];
      }
      // pairs q = 0..8: (1,2) x, (3,4) y, (5,6) z, (7,8) xy+, (9,10) xy-, (11,12) xz+, (13,14) xz-, (15,16) yz+, (17,18) yz-
      float sh[9], dhh[9], sl[9], dll[9], sg[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int a = 2 * q + 1, c = 2 * q + 2;
        sh[q] = h[a] + h[c];
        dhh[q] = h[a] - h[c];
        sl[q] = l[a] + l[c];
        dll[q] = l[a] - l[c];
        sg[q] = g[a] + g[c];
      }
      const float dh = h[0] + (((sh[0] + sh[1]) + (sh[2] + sh[3])) + ((sh[4] + sh[5]) + ((sh[6] + sh[7]) + sh[8])));
      const float dl = l[0] + (((sl[0] + sl[1]) + (sl[2] + sl[3])) + ((sl[4] + sl[5]) + ((sl[6] + sl[7]) + sl[8])));
      // sum c g as hi + lo
      const float jxh = (dhh[0] + (dhh[3] + dhh[4])) + (dhh[5] + dhh[6]);
      const float jyh = (dhh[1] + (dhh[3] - dhh[4])) + (dhh[7] + dhh[8]);
      const float jzh = (dhh[2] + (dhh[5] - dhh[6])) + (dhh[7] - dhh[8]);
      const float jxl = (dll[0] + (dll[3] + dll[4])) + (dll[5] + dll[6]);
      const float jyl = (dll[1] + (dll[3] - dll[4])) + (dll[7] + dll[8]);
      const float jzl = (dll[2] + (dll[5] - dll[6])) + (dll[7] - dll[8]);
      const float drho = dh + dl;
      const float gsum = g[0] + (((sg[0] + sg[1]) + (sg[2] + sg[3])) + ((sg[4] + sg[5]) + ((sg[6] + sg[7]) + sg[8])));
      // sum (3 c_a c_b - delta_ab) g: 3 (sum of the pairs with c_a != 0) - sum g
      const float hxx = 3.0f * (sg[0] + ((sg[3] + sg[4]) + (sg[5] + sg[6]))) - gsum;
      const float hyy = 3.0f * (sg[1] + ((sg[3] + sg[4]) + (sg[7] + sg[8]))) - gsum;
      const float hzz = 3.0f * (sg[2] + ((sg[5] + sg[6]) + (sg[7] + sg[8]))) - gsum;
      const float hxy = 3.0f * (sg[3] - sg[4]);
      const float hxz = 3.0f * (sg[5] - sg[6]);
      const float hyz = 3.0f * (sg[7] - sg[8]);

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

      // Output.  For a pair (a, opp(a)) with velocity c:
      //   g'/w = [drho + 3 c.J] + rho (4.5 (c.u)^2 - 1.5 u.u) + (1 - 1/tau) 4.5 Q:Pi_neq (+ force terms)
      // the bracket is exact from the hi parts (big, odd in c); everything else is
      // small and split into an even part E and an odd part O.  w_i is applied as
      // w_hi S + w_lo S (one rounding, no systematic bias from rounding w_i).
      const float omhw = FORCE ? s * itau : 0.0f;         // 1 - 1/(2 tau)
      const float uF = FORCE ? ux * p.fx + uy * p.fy + uz * p.fz : 0.0f;
      const float base_e = dl - rho * uu15;
      float o[kQ];
      {
        // rest population: c = 0
        float e0 = base_e + omw45 * (-tr3);
        if (FORCE) e0 += -3.0f * omhw * uF;
        o[0] = wmul(0, dh + e0);
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int a = 2 * q + 1;
        const int cx = CX[a], cy = CY[a], cz = CZ[a];
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
        o[a] = wmul(a, (dh + Oh) + (E + Ol));
        o[a + 1] = wmul(a + 1, (dh - Oh) + (E - Ol));
      }
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
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

    if (active) {
#pragma unroll
      for (int i = 0; i < kQ; ++i)
        Vec::store(out[i], rout, v_here, static_cast<unsigned>(i) * pop_bytes + row_here);
    }
  }

  // one flag write per wave
  if (__any(bad && active && wave_live)) {
    if (lane == 0) atomicOr(p.flag, kFlagDensity);
  }

  if (STATS) {
    // per-(x, y) sums over the block's z range: registers, then the wz waves in LDS
    extern __shared__ float red[];             // [wz][9][64 wx V]
    const int tx = threadIdx.x, bx = 64 * p.wx * V;
    if (p.wz > 1) {
#pragma unroll
      for (int q = 0; q < 9; ++q)
#pragma unroll
        for (int k = 0; k < V; ++k) red[(wz * 9 + q) * bx + tx * V + k] = acc[q][k];
      __syncthreads();
    }
    if (wz == 0 && active && wave_live) {
      const long long sstride = (long long)ny * nx;
      double* st = p.stats + (long long)slot * 9 * sstride + (long long)y * nx + x0;
#pragma unroll
      for (int q = 0; q < 9; ++q)
#pragma unroll
        for (int k = 0; k < V; ++k) {
          float v = acc[q][k];
          for (int w = 1; w < p.wz; ++w) v += red[(w * 9 + q) * bx + tx * V + k];
          st[q * sstride + k] += static_cast<double>(v);
        }
    }
  }
}

__global__ void fill_zero_kernel(uint4* p, unsigned long long n16) {
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, unsigned long long n16) {
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
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

// Public element e of [19][NZ][NY][NX] -> stored element of [NZ][19][NY][NX].
__device__ __forceinline__ long long stored_index(long long e, int nz, long long plane2d, int* pop) {
  const long long plane = static_cast<long long>(nz) * plane2d;
  const int i = static_cast<int>(e / plane);
  const long long r = e - i * plane;              // z * plane2d + (y, x)
  const long long z = r / plane2d;
  *pop = i;
  return (z * kQ + i) * plane2d + (r - z * plane2d);
}

template <class Codec>
__global__ void export_f_kernel(const typename Codec::storage* g, long long offset, long long count, int nz,
                                long long plane2d, double* out) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride) {
    int i;
    const long long at = stored_index(offset + k, nz, plane2d, &i);
    out[k] = weight_d(i) + static_cast<double>(Codec::decode(g[at]));
  }
}

template <class Codec>
__global__ void export_planes_kernel(const typename Codec::storage* g, int nx, int ny, int nz, int x0, int w,
                                     double* out) {
  const long long count = (long long)kQ * nz * ny * w;
  const long long plane2d = (long long)nx * ny;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride) {
    const int xx = static_cast<int>(k % w);
    const long long r = k / w;                    // (i, z, y)
    const int i = static_cast<int>(r / ((long long)nz * ny));
    const long long zy = r % ((long long)nz * ny);
    const long long z = zy / ny, y = zy % ny;
    out[k] = weight_d(i) + static_cast<double>(Codec::decode(g[(z * kQ + i) * plane2d + y * nx + x0 + xx]));
  }
}

template <class Codec>
__global__ void import_f_kernel(const double* f, long long offset, long long count, int nz, long long plane2d,
                                typename Codec::storage* g) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride) {
    int i;
    const long long at = stored_index(offset + k, nz, plane2d, &i);
    g[at] = Codec::encode(static_cast<float>(f[k] - weight_d(i)));
  }
}

// f = f_eq(rho = 1, u) (eq. local_eq) from a velocity field u[3][NZ][NY][NX]
// in lattice units, computed in FP64 and rounded once to the store type.
template <class Codec>
__global__ void equilibrium_kernel(const double* u, int nx, int ny, int nz, typename Codec::storage* g) {
  const long long plane2d = (long long)nx * ny;
  const long long cells = plane2d * nz;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += stride) {
    const double ux = u[c], uy = u[cells + c], uz = u[2 * cells + c];
    const double uu = ux * ux + uy * uy + uz * uz;
    const long long z = c / plane2d, yx = c - z * plane2d;
    for (int i = 0; i < kQ; ++i) {
      const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
      g[(z * kQ + i) * plane2d + yx] = Codec::encode(static_cast<float>(weight_d(i) * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu)));
    }
  }
}

// Velocity of the collision at the probe cells, recovered from the
// post-collision state: collision keeps rho and returns sum c f = rho u + F/2
// (regularized operator with J_neq = -F/2 plus the Guo source).  FP64 sums.
template <class Codec>
__global__ void probe_kernel(ProbeParams p) {
  const int k = threadIdx.x;
  if (k >= p.n) return;
  const auto* g = static_cast<const typename Codec::storage*>(p.g);
  const long long base = (long long)p.xyz[k][2] * kQ * p.plane2d + (long long)p.xyz[k][1] * p.nx + p.xyz[k][0];
  double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for (int i = 0; i < kQ; ++i) {
    const double f = weight_d(i) + static_cast<double>(Codec::decode(g[base + i * p.plane2d]));
    rho += f;
    jx += CX[i] * f;
    jy += CY[i] * f;
    jz += CZ[i] * f;
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

template <class Codec, int V>
hipError_t launch_step_v(const StepParams& p, bool stats, hipStream_t s) {
  const dim3 block(64 * p.wx, p.wz);
  const dim3 grid(p.nblocks);
  const size_t lds = (stats && p.wz > 1) ? sizeof(float) * 9 * 64 * V * p.wx * p.wz : 0;
  if (p.has_force) {
    if (stats) step_kernel<Codec, V, true, true><<<grid, block, lds, s>>>(p);
    else step_kernel<Codec, V, false, true><<<grid, block, 0, s>>>(p);
  } else {
    if (stats) step_kernel<Codec, V, true, false><<<grid, block, lds, s>>>(p);
    else step_kernel<Codec, V, false, false><<<grid, block, 0, s>>>(p);
  }
  return hipGetLastError();
}

template <class Codec>
hipError_t launch_step_codec(const StepParams& p, bool stats, hipStream_t s) {
  if (p.wx < 1 || p.wz < 1 || p.wx * p.wz > kMaxWavesPerBlock) return hipErrorInvalidValue;
  if (p.vec < 1 || p.nx % p.vec != 0) return hipErrorInvalidValue;
  switch (p.vec) {
    case 1: return launch_step_v<Codec, 1>(p, stats, s);
    case 2: return launch_step_v<Codec, 2>(p, stats, s);
    case 4: return launch_step_v<Codec, 4>(p, stats, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_step(const StepParams& p, int store, bool stats, hipStream_t s) {
  switch (store) {
    case 0: return launch_step_codec<CodecF32>(p, stats, s);
    case 1: return launch_step_codec<CodecF16>(p, stats, s);
    case 2: return launch_step_codec<CodecBF16>(p, stats, s);
    default: return hipErrorInvalidValue;
  }
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

hipError_t launch_sponge(float* sponge, int nx, int cells, double K, double pw, hipStream_t s) {
  sponge_kernel<<<(nx + 255) / 256, 256, 0, s>>>(sponge, nx, cells, K, pw);
  return hipGetLastError();
}

hipError_t launch_export_f(const void* g, int store, long long offset, long long count, int nz, long long plane2d,
                           double* out, hipStream_t s) {
  const int grid = grid_for(static_cast<unsigned long long>(count), 256);
  switch (store) {
    case 0: export_f_kernel<CodecF32><<<grid, 256, 0, s>>>(static_cast<const float*>(g), offset, count, nz, plane2d, out); break;
    case 1: export_f_kernel<CodecF16><<<grid, 256, 0, s>>>(static_cast<const unsigned short*>(g), offset, count, nz, plane2d, out); break;
    case 2: export_f_kernel<CodecBF16><<<grid, 256, 0, s>>>(static_cast<const unsigned short*>(g), offset, count, nz, plane2d, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_export_planes(const void* g, int store, int nx, int ny, int nz, int x0, int x1, double* out,
                               hipStream_t s) {
  const int w = x1 - x0;
  const int grid = grid_for(static_cast<unsigned long long>(kQ) * nz * ny * w, 256);
  switch (store) {
    case 0: export_planes_kernel<CodecF32><<<grid, 256, 0, s>>>(static_cast<const float*>(g), nx, ny, nz, x0, w, out); break;
    case 1: export_planes_kernel<CodecF16><<<grid, 256, 0, s>>>(static_cast<const unsigned short*>(g), nx, ny, nz, x0, w, out); break;
    case 2: export_planes_kernel<CodecBF16><<<grid, 256, 0, s>>>(static_cast<const unsigned short*>(g), nx, ny, nz, x0, w, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_import_f(const double* f, int store, long long offset, long long count, int nz, long long plane2d,
                           void* g, hipStream_t s) {
  const int grid = grid_for(static_cast<unsigned long long>(count), 256);
  switch (store) {
    case 0: import_f_kernel<CodecF32><<<grid, 256, 0, s>>>(f, offset, count, nz, plane2d, static_cast<float*>(g)); break;
    case 1: import_f_kernel<CodecF16><<<grid, 256, 0, s>>>(f, offset, count, nz, plane2d, static_cast<unsigned short*>(g)); break;
    case 2: import_f_kernel<CodecBF16><<<grid, 256, 0, s>>>(f, offset, count, nz, plane2d, static_cast<unsigned short*>(g)); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_equilibrium(const double* u, int store, int nx, int ny, int nz, void* g, hipStream_t s) {
  const int grid = grid_for(static_cast<unsigned long long>(nx) * ny * nz, 256);
  switch (store) {
    case 0: equilibrium_kernel<CodecF32><<<grid, 256, 0, s>>>(u, nx, ny, nz, static_cast<float*>(g)); break;
    case 1: equilibrium_kernel<CodecF16><<<grid, 256, 0, s>>>(u, nx, ny, nz, static_cast<unsigned short*>(g)); break;
    case 2: equilibrium_kernel<CodecBF16><<<grid, 256, 0, s>>>(u, nx, ny, nz, static_cast<unsigned short*>(g)); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_probes(const ProbeParams& p, int store, hipStream_t s) {
  if (p.n < 1 || p.n > kMaxProbes) return hipErrorInvalidValue;
  switch (store) {
    case 0: probe_kernel<CodecF32><<<1, 64, 0, s>>>(p); break;
    case 1: probe_kernel<CodecF16><<<1, 64, 0, s>>>(p); break;
    case 2: probe_kernel<CodecBF16><<<1, 64, 0, s>>>(p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace stglbm
