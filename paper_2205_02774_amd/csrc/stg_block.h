// One block of the STG inlet plane (eqs. aux_vec, psu, v_fluc, u_phys,
// u_transfer), shared by the plane kernel (inlet_kernels.hip) and the trailing
// blocks of the stream-collide launch (lattice_step.h), which make the plane of
// a later step while the launch's last lattice blocks finish.
//
// v' = sqrt 6 sum_n sqrt(q^n) sigma^n cos(psi_n), u' = a v', u_bc = (U + u')
// c_t / c_x.  The phase splits into a row part (FP64 per row, mode and step,
// kept as the FP32 phasor P = sqrt 6 sqrt(q) exp(i psi_row)) and the spanwise
// phasor B = exp(i k d_z z) of the precomputed table, so cos(psi) =
// Re(P B) / |P|.  The block covers kRows rows x 64 spanwise nodes of one plane;
// wave w < kStgWaves sums the modes n = w mod kStgWaves for all its rows, in
// increasing n, so each B loaded serves kRows rows; the partial sums meet in
// LDS in wave order.  A node's value therefore depends neither on kRows, nor
// on kChunk (the modes staged per pass, a multiple of kStgWaves), nor on
// kInFlight (the spanwise phasor loads a wave keeps in flight), nor on which
// launch makes it: every term is the same explicit chain of multiplies and
// FMAs.  Waves w >= kStgWaves of a larger block only join the barriers.
#pragma once
#include "stglbm_internal.h"

namespace stglbm {
namespace {

// LDS bytes of a block: the staging of a pass (time phasors, sigma, row
// phasors) and the partial sums share the space.
template <int kRows, int kChunk>
constexpr int stg_block_lds() {
  const int stage = kChunk * 16 + kChunk * 16 + kRows * kChunk * 8;
  const int red = kStgWaves * 3 * kRows * 64 * 4;
  return stage > red ? stage : red;
}

// One mode's term for kRows rows: c = Re(P B) (scaled cos of the full phase),
// v += sigma c.
template <int kRows, int kChunk>
__device__ __forceinline__ void stg_term(float (&v)[kRows][3], const float4 S, const float2 (*P)[kChunk], int m,
                                         const float2 B) {
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const float2 Pm = P[r][m];
    const float c = __builtin_fmaf(Pm.x, B.x, -(Pm.y * B.y));
    v[r][0] = __builtin_fmaf(S.x, c, v[r][0]);
    v[r][1] = __builtin_fmaf(S.y, c, v[r][1]);
    v[r][2] = __builtin_fmaf(S.z, c, v[r][2]);
  }
}

template <int kRows, int kChunk, int kInFlight>
__device__ __forceinline__ void stg_plane_block(const StgParams& p, int plane, int zblk, int rowblk, int lane,
                                                int w, char* smem) {
  static_assert(kChunk % kStgWaves == 0, "a pass must hold whole rounds of the waves' modes");
  const bool work = w < kStgWaves;
  const int tid = w * 64 + lane;
  const int j0 = rowblk * kRows;
  const int z = zblk * 64 + lane;
  const double tphase = p.tphase[plane];
  const int zc = z < p.nz ? z : p.nz - 1;
  double2* G = reinterpret_cast<double2*>(smem);
  float4* SG = reinterpret_cast<float4*>(smem + kChunk * 16);
  float2 (*P)[kChunk] = reinterpret_cast<float2 (*)[kChunk]>(smem + kChunk * 32);
  float (*red)[3 * kRows][64] = reinterpret_cast<float (*)[3 * kRows][64]>(smem);
  float v[kRows][3];
#pragma unroll
  for (int r = 0; r < kRows; ++r) v[r][0] = v[r][1] = v[r][2] = 0.f;
  for (int base = 0; base < p.n_modes; base += kChunk) {
    const int cnt = min(kChunk, p.n_modes - base);
    // time part of the phase, per mode: exp(i 2 pi d_x (x_in - U_b t) / L_e)
    if (work) {
      for (int m = tid; m < cnt; m += 64 * kStgWaves) {
        double sn, cs;
        sincos(p.modes[(long long)(base + m) * kModeFields + 1] * tphase, &sn, &cs);
        G[m] = make_double2(cs, sn);
        SG[m] = p.sig[base + m];
      }
    }
    __syncthreads();
    // P = sqrt 6 sqrt(q) exp(i psi_row) of the full row part: the stored
    // time-independent phasor times the time part, in FP64, rounded once
    // (0 past the last row)
    if (work) {
      for (int e = tid; e < kRows * cnt; e += 64 * kStgWaves) {
        const int r = e / cnt, m = e - r * cnt;
        const int j = j0 + r;
        float2 ph = make_float2(0.f, 0.f);
        if (j < p.ny) {
          const double2 a = p.arow[(long long)j * p.n_modes + base + m];
          const double2 g = G[m];
          ph = make_float2(static_cast<float>(__builtin_fma(a.x, g.x, -(a.y * g.y))),
                           static_cast<float>(__builtin_fma(a.x, g.y, a.y * g.x)));
        }
        P[r][m] = ph;
      }
    }
    __syncthreads();
    if (work) {
      const float2* bz = p.bz + (long long)base * p.nz + zc;
      const long long step = (long long)kStgWaves * p.nz;
      int m = w;
      for (; m + (kInFlight - 1) * kStgWaves < cnt; m += kInFlight * kStgWaves) {
        float2 Bs[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) Bs[u] = bz[(long long)m * p.nz + u * step];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) stg_term<kRows, kChunk>(v, SG[m + u * kStgWaves], P, m + u * kStgWaves, Bs[u]);
      }
      for (; m < cnt; m += kStgWaves) stg_term<kRows, kChunk>(v, SG[m], P, m, bz[(long long)m * p.nz]);
    }
    __syncthreads();
  }
  if (work) {
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
      const double u0 = row[0] + a11 * vs[0];
      const double u1 = row[1] + a21 * vs[0] + a22 * vs[1];
      const double u2 = row[2] + a31 * vs[0] + a32 * vs[1] + a33 * vs[2];
      float* o = p.out + 3 * ((long long)plane * p.ny * p.nz + (long long)j * p.nz + z);
      o[0] = static_cast<float>(u0 * p.conv);
      o[1] = static_cast<float>(u1 * p.conv);
      o[2] = static_cast<float>(u2 * p.conv);
    }
  }
}

}  // namespace
}  // namespace stglbm
