// One block of the STG inlet plane (eqs. aux_vec, psu, v_fluc, u_phys,
// u_transfer), shared by the plane kernel (inlet_kernels.hip) and the trailing
// blocks of the stream-collide launch (lattice_step.h), which make the plane of
// a later step while the launch's last lattice blocks finish.
//
// v' = sqrt 6 sum_n sqrt(q^n) sigma^n cos(psi_n), u' = a v', u_bc = (U + u')
// c_t / c_x.  The phase splits into a row part (FP64 per row, mode and step,
// kept as the FP32 phasor P = sqrt 6 sqrt(q) exp(i psi_row)) and the spanwise
// phasor B = exp(i k d_z z) of the precomputed table, so cos(psi) =
// Re(P B) / |P|.  The row phasors of a plane sit in a table [mode][row]
// (stg_time_phase_kernel makes those of 16 steps at a time), so each wave reads
// the P and sigma of its mode with scalar loads: they are the same for all its
// lanes and feed the FMAs from scalar registers, and only the spanwise phasor
// is a vector load.  The block covers kRows rows x 64 spanwise nodes of one
// plane; wave w < kStgWaves sums the modes n = w mod kStgWaves for all its
// rows, in increasing n, so each B loaded serves kRows rows; the partial sums
// meet in LDS in wave order.  A node's value therefore depends neither on
// kRows, nor on kInFlight (the spanwise phasor loads a wave keeps in flight),
// nor on which launch makes it: every term is the same explicit chain of
// multiplies and FMAs.  Waves w >= kStgWaves of a larger block only join the
// barrier.
#pragma once
#include "stglbm_internal.h"

namespace stglbm {
namespace {

// LDS bytes of a block: the waves' partial sums.
template <int kRows>
constexpr int stg_block_lds() {
  return kStgWaves * 3 * kRows * 64 * 4;
}

// P = a g for the time-independent row phasor a and the time factor g, in
// FP64, rounded once to FP32.
__device__ __forceinline__ float2 stg_row_phasor(const double2 a, const double2 g) {
  return make_float2(static_cast<float>(__builtin_fma(a.x, g.x, -(a.y * g.y))),
                     static_cast<float>(__builtin_fma(a.x, g.y, a.y * g.x)));
}

// One mode's term for kRows rows: c = Re(P B) (scaled cos of the full phase),
// v += sigma c.
template <int kRows>
__device__ __forceinline__ void stg_term(float (&v)[kRows][3], const float4 S, const float2* __restrict__ P,
                                         const float2 B) {
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const float2 Pm = P[r];
    const float c = __builtin_fmaf(Pm.x, B.x, -(Pm.y * B.y));
    v[r][0] = __builtin_fmaf(S.x, c, v[r][0]);
    v[r][1] = __builtin_fmaf(S.y, c, v[r][1]);
    v[r][2] = __builtin_fmaf(S.z, c, v[r][2]);
  }
}

template <int kRows, int kInFlight>
__device__ __forceinline__ void stg_plane_block(const StgParams& p, int plane, int zblk, int rowblk, int lane,
                                                int w, char* smem) {
  w = __builtin_amdgcn_readfirstlane(w);
  const bool work = w < kStgWaves;
  const int j0 = rowblk * kRows;
  const int z = zblk * 64 + lane;
  const int zc = z < p.nz ? z : p.nz - 1;
  float (*red)[3 * kRows][64] = reinterpret_cast<float (*)[3 * kRows][64]>(smem);
  float v[kRows][3];
#pragma unroll
  for (int r = 0; r < kRows; ++r) v[r][0] = v[r][1] = v[r][2] = 0.f;
  if (work) {
    // P of this plane, [mode][row]: the block's kRows rows of mode m at P + m * rows
    const int prow = p.ptab_rows;
    const float2* __restrict__ P = p.ptab + (long long)p.pslot[plane] * p.n_modes * prow + j0;
    const float4* __restrict__ sig = p.sig;
    const float2* __restrict__ bz = p.bz + zc;
    const long long step = (long long)kStgWaves * p.nz;
    int m = w;
    for (; m + (kInFlight - 1) * kStgWaves < p.n_modes; m += kInFlight * kStgWaves) {
      float2 Bs[kInFlight];
#pragma unroll
      for (int u = 0; u < kInFlight; ++u) Bs[u] = bz[(long long)m * p.nz + u * step];
#pragma unroll
      for (int u = 0; u < kInFlight; ++u) {
        const int mm = m + u * kStgWaves;
        stg_term<kRows>(v, sig[mm], P + (long long)mm * prow, Bs[u]);
      }
    }
    for (; m < p.n_modes; m += kStgWaves) stg_term<kRows>(v, sig[m], P + (long long)m * prow, bz[(long long)m * p.nz]);
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) red[w][3 * r + c][lane] = v[r][c];
  }
  __syncthreads();
  // one thread per (row, node) of the block: waves 0 .. kRows-1 take one row each
  if (w < kRows) {
    const int j = j0 + w;
    if (j < p.ny && z < p.nz) {
      float vs[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float acc = red[0][3 * w + c][lane];
#pragma unroll
        for (int k = 1; k < kStgWaves; ++k) acc += red[k][3 * w + c][lane];
        vs[c] = acc;
      }
      const double* row = p.rows + (long long)j * kRowFields;
      const double a11 = row[11], a21 = row[12], a22 = row[13], a31 = row[14], a32 = row[15], a33 = row[16];
      // u = U + a v', the terms added left to right, each as one FMA
      const double u0 = __builtin_fma(a11, vs[0], row[0]);
      const double u1 = __builtin_fma(a22, vs[1], __builtin_fma(a21, vs[0], row[1]));
      const double u2 = __builtin_fma(a33, vs[2], __builtin_fma(a32, vs[1], __builtin_fma(a31, vs[0], row[2])));
      float* o = p.out + 3 * ((long long)plane * p.ny * p.nz + (long long)j * p.nz + z);
      o[0] = static_cast<float>(u0 * p.conv);
      o[1] = static_cast<float>(u1 * p.conv);
      o[2] = static_cast<float>(u2 * p.conv);
    }
  }
}

}  // namespace
}  // namespace stglbm
