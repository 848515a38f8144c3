// HIP kernels of the psoam hot path for gfx950 (MI355X).
//
//  switch_fwd*  b = S c           photo-switching matrix per voxel (eq. Sij-detailed)
//  band16/32    y = H b, r = H b - p, or c = S^T H^T r
//               (acoustic operator, Sec. 2.1.4 / 2.2.3; block-diagonal over
//               pulses as W_tot, eq. acoustic-full-forward)
//  pack_r*      y -> padded operand of H^T
//  tv_*         one step of the dual iteration of the TV prox (Alg. alg:prox-inner)
//  prox_l1      soft threshold (+ x >= 0)
//  reductions   deterministic FP64 two-stage sums (objective, norms, power iteration)
//
// Matrix-core mapping of the band contraction.  For one output tile of 16
// rows (16 samples t for H, 16 depths z for H^T) and one position, the
// contraction runs over (lateral offset, contracted sample) pairs whose band
// entry is nonzero in the tile.  These are packed 4 groups per chunk; a group
// is an 8-sample octet (16-bit inputs, v_mfma_f32_16x16x32_{bf16,f16}) or a
// single sample (FP32 inputs, v_mfma_f32_16x16x4_f32) at one lateral offset.
// The 16 columns of the instruction are 16 pulses: the band block (operand A)
// is shared by every pulse and every position, so each wave loads it once per
// chunk and reuses it for kPosPerWave positions x (Kp/16) pulse blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "psoam_internal.h"

namespace psoam {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// word 3 of a raw buffer resource on CDNA (32-bit data format, no swizzle)
constexpr int kBufWord3 = 0x00020000;
// s_waitcnt operand: vmcnt(0), expcnt and lgkmcnt left at their maxima
constexpr int kVmcnt0 = 0x0F70;

template <int PREC>
struct Half;

template <>
struct Half<PSOAM_BF16> {
  using E = __bf16;
  using V = bf16x8;
  using V4 = bf16x4;
  static constexpr float scale = 1.0f;
  static __device__ __forceinline__ f32x4 mma(V a, V b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Half<PSOAM_FP16> {
  using E = _Float16;
  using V = f16x8;
  using V4 = f16x4;
  static constexpr float scale = kFp16Scale;
  static __device__ __forceinline__ f32x4 mma(V a, V b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// --------------------------------------------------------------------------
// photo-switching coefficient S_v[k][s] (eq. final-H with the rate written
// per pulse as phi^gamma / tau)
// --------------------------------------------------------------------------
__device__ __forceinline__ float scoef(const SwitchParams& sw, float phi, int k, int s) {
  if (sw.diag) return k == s ? phi : 0.0f;
  const float pg = (sw.gamma == 0.0f) ? 1.0f : powf(phi, sw.gamma);
  return phi * (sw.a[s] + sw.b[s] * expf(-(float)k * pg * sw.inv_tau[s]));
}

// the same coefficient from the depth-fastest table [K][S][Nz] (kernels whose
// consecutive lanes are consecutive depths read it coalesced)
__device__ __forceinline__ float coef_zt(const SwitchParams& sw, const float* __restrict__ phi,
                                         const float* __restrict__ stab_t, int nz, size_t col,
                                         int z, int k, int s) {
  if (stab_t) return stab_t[((size_t)k * sw.ns + s) * nz + z];
  return scoef(sw, phi[col + z], k, s);
}

__device__ __forceinline__ float coef_at(const SwitchParams& sw, const float* __restrict__ phi,
                                         const float* __restrict__ stab, int kp, size_t col,
                                         int z, int k, int s) {
  if (stab) return stab[((size_t)z * kp + k) * sw.ns + s];
  return scoef(sw, phi[col + z], k, s);
}

// b[k][y][x][z] = sum_s S[k][s] c[s][y][x][z] into the 16-bit octet operand.
// One thread per (y, x, octet, pulse); pulses beyond K are written as zeros.
// With `vec` (Nz a multiple of 8, c 16-byte aligned, the per-depth octet
// table [Lz/8][S][Kp][8] present) a species' octet and its eight
// coefficients arrive in four 16-byte loads issued together, instead of a
// chain of guarded scalar loads; the sums are the same, in the same order.
template <int PREC, bool SPLIT>
__global__ __launch_bounds__(256) void switch_fwd16(const float* __restrict__ c,
                                                    const float* __restrict__ phi,
                                                    const float* __restrict__ stab,
                                                    const float* __restrict__ stab_o, int vec,
                                                    const float* __restrict__ f16, SwitchParams sw,
                                                    typename Half<PREC>::E* __restrict__ bq,
                                                    typename Half<PREC>::E* __restrict__ bq_lo,
                                                    int ny, int nx, int nz, int zo_n, int kp,
                                                    int xp, int r, size_t ps,
                                                    const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  using H = Half<PREC>;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)ny * nx * zo_n * kp;
  if (tid >= total) return;
  int k, zo, x, y;
  if (total <= 0xffffffffu) {  // 32-bit index arithmetic where it fits
    unsigned rest = (unsigned)tid;
    k = (int)(rest % (unsigned)kp);
    rest /= (unsigned)kp;
    zo = (int)(rest % (unsigned)zo_n);
    rest /= (unsigned)zo_n;
    x = (int)(rest % (unsigned)nx);
    y = (int)(rest / (unsigned)nx);
  } else {
    size_t rest = tid / kp;
    k = (int)(tid % kp);
    zo = (int)(rest % zo_n);
    rest /= zo_n;
    x = (int)(rest % nx);
    y = (int)(rest / nx);
  }
  float b[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) b[j] = 0.0f;
  if (k < sw.nk && vec) {
    const size_t col = ((size_t)y * nx + x) * nz + (size_t)zo * 8;
    const int s0 = sw.diag ? k : 0, s1 = sw.diag ? (k < sw.ns ? k + 1 : k) : sw.ns;
    for (int s = s0; s < s1; ++s) {
      const f32x4* cs = (const f32x4*)(c + (size_t)s * ny * nx * nz + col);
      const f32x4* ws = (const f32x4*)(stab_o + (((size_t)zo * sw.ns + s) * kp + k) * 8);
      const f32x4 c0 = cs[0], c1 = cs[1], w0 = ws[0], w1 = ws[1];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        b[j] += w0[j] * c0[j];
        b[4 + j] += w1[j] * c1[j];
      }
    }
  } else if (k < sw.nk) {
    const size_t col = ((size_t)y * nx + x) * nz;
    // diagonal switching: only species k contributes
    const int s0 = sw.diag ? k : 0, s1 = sw.diag ? (k < sw.ns ? k + 1 : k) : sw.ns;
    for (int s = s0; s < s1; ++s) {
      const float* cs = c + (size_t)s * ny * nx * nz + col;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int z = zo * 8 + j;
        if (z < nz) b[j] += coef_at(sw, phi, stab, kp, col, z, k, s) * cs[z];
      }
    }
  }
  // operand scale: the per-call power of two of FP16 plans (1 for BF16)
  const float sc = f16 ? f16[0] : H::scale;
  typename H::V hi, lo;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float v = b[j] * sc;
    hi[j] = (typename H::E)v;
    lo[j] = (typename H::E)(v - (float)hi[j]);
  }
  const size_t o = ((size_t)(y + r) * xp + (x + r)) * ps + ((size_t)zo * kp + k) * 8;
  *(typename H::V*)(bq + o) = hi;
  if constexpr (SPLIT) *(typename H::V*)(bq_lo + o) = lo;
}

// FP32 operand [Yp][Xp][Nz][Kp]: one thread per (y, x, z, pulse), pulses fastest.
__global__ __launch_bounds__(256) void switch_fwd32(const float* __restrict__ c,
                                                    const float* __restrict__ phi,
                                                    const float* __restrict__ stab,
                                                    SwitchParams sw, float* __restrict__ bq,
                                                    int ny, int nx, int nz, int kp, int xp,
                                                    int r, size_t ps, const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)ny * nx * nz * kp;
  if (tid >= total) return;
  const int k = (int)(tid % kp);
  size_t rest = tid / kp;
  const int z = (int)(rest % nz);
  rest /= nz;
  const int x = (int)(rest % nx);
  const int y = (int)(rest / nx);
  float b = 0.0f;
  if (k < sw.nk) {
    const size_t col = ((size_t)y * nx + x) * nz;
    const int s0 = sw.diag ? k : 0, s1 = sw.diag ? (k < sw.ns ? k + 1 : k) : sw.ns;
    for (int s = s0; s < s1; ++s)
      b += coef_at(sw, phi, stab, kp, col, z, k, s) * c[(size_t)s * ny * nx * nz + col + z];
  }
  bq[((size_t)(y + r) * xp + (x + r)) * ps + (size_t)z * kp + k] = b;
}

// y[k][y][x][t] -> 16-bit octet operand of H^T at the padded position,
// rq[pos][t/8][k][8].  One block per position, in chunks of 16 pulses x 16
// octets transposed through LDS: a thread reads 8 consecutive samples of one
// pulse (16 threads cover 512 contiguous bytes of a pulse row) and, after the
// barrier, writes the 16-byte octet of (octet t/16, pulse t%16), so 16
// consecutive threads write 256 contiguous bytes.
template <int PREC, bool SPLIT>
__global__ __launch_bounds__(256) void pack_r16(const float* __restrict__ yin,
                                                typename Half<PREC>::E* __restrict__ rq,
                                                typename Half<PREC>::E* __restrict__ rq_lo,
                                                int nk, int ny, int nx, int nt, int to_n,
                                                int kp, int xp, int r, size_t ps, int vec4,
                                                int tsh, const float* __restrict__ f16,
                                                const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  using H = Half<PREC>;
  using V = typename H::V;
  const float sc = f16 ? f16[2] : H::scale;   // operand scale (FP16: per call)
  __shared__ V t_hi[256];
  __shared__ V t_lo[SPLIT ? 256 : 1];
  const int pos = blockIdx.x;
  const int y = pos / nx, x = pos % nx;
  const size_t o_pos = ((size_t)(y + r) * xp + (x + r)) * ps;
  const int tid = threadIdx.x;
  const int a = tid >> 4, c = tid & 15;
  for (int kc = 0; kc < kp; kc += 16) {
    for (int oc = 0; oc < to_n; oc += 16) {
      // read: pulse kc + a, octet oc + c
      {
        const int k = kc + a, to = oc + c;
        V hi, lo;
        if (k < nk && to < to_n) {
          // octet `to` holds samples to*8 - tsh .. to*8 - tsh + 7
          const int tb = to * 8 - tsh;
          const float* row = yin + (((size_t)k * ny + y) * nx + x) * nt;
          float v[8];
          if (vec4 && tb >= 0 && tb + 7 < nt) {
            const f32x4 v0 = *(const f32x4*)(row + tb), v1 = *(const f32x4*)(row + tb + 4);
            v[0] = v0[0]; v[1] = v0[1]; v[2] = v0[2]; v[3] = v0[3];
            v[4] = v1[0]; v[5] = v1[1]; v[6] = v1[2]; v[7] = v1[3];
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (tb + j >= 0 && tb + j < nt) ? row[tb + j] : 0.0f;
          }
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const float w = v[j] * sc;
            hi[j] = (typename H::E)w;
            lo[j] = (typename H::E)(w - (float)hi[j]);
          }
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            hi[j] = (typename H::E)0.0f;
            lo[j] = (typename H::E)0.0f;
          }
        }
        t_hi[c * 16 + a] = hi;
        if constexpr (SPLIT) t_lo[c * 16 + a] = lo;
      }
      __syncthreads();
      // write: octet oc + a, pulse kc + c
      {
        const int to = oc + a, k = kc + c;
        if (to < to_n) {
          const size_t o = o_pos + ((size_t)to * kp + k) * 8;
          *(V*)(rq + o) = t_hi[a * 16 + c];
          if constexpr (SPLIT) *(V*)(rq_lo + o) = t_lo[a * 16 + c];
        }
      }
      __syncthreads();
    }
  }
}

// y[k][pos][t] -> rq[pos][t][k] (FP32), transposed through LDS, one block per position.
__global__ __launch_bounds__(256) void pack_r32(const float* __restrict__ yin,
                                                float* __restrict__ rq, int nk, int ny, int nx,
                                                int nt, int lt, int kp, int xp, int r,
                                                size_t ps, const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  __shared__ float tile[64][65];
  const int pos = blockIdx.x;
  const int y = pos / nx, x = pos % nx;
  float* dst = rq + ((size_t)(y + r) * xp + (x + r)) * ps;
  for (int k0 = 0; k0 < kp; k0 += 64) {
    for (int t0 = 0; t0 < lt; t0 += 64) {
      for (int i = threadIdx.x; i < 64 * 64; i += 256) {
        const int kk = i / 64, tt = i % 64;
        const int k = k0 + kk, t = t0 + tt;
        tile[kk][tt] = (k < nk && t < nt) ? yin[(((size_t)k * ny + y) * nx + x) * nt + t] : 0.0f;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < 64 * 64; i += 256) {
        const int tt = i / 64, kk = i % 64;
        const int k = k0 + kk, t = t0 + tt;
        if (k < kp && t < lt) dst[(size_t)t * kp + k] = tile[kk][tt];
      }
      __syncthreads();
    }
  }
}

// --------------------------------------------------------------------------
// band contraction
// --------------------------------------------------------------------------
struct BandArgs {
  const void* q;
  const void* q_lo;
  const int* start;
  const int* off;
  const void* a;
  const void* a_lo;
  int n_mtiles, n_mblk, ny, nx, nxb, m_rows, xp;
  size_t ps;
  int nk, kp;
  int half;          // staged kernels: the last 16-pulse block runs in half form
  float inv_scale;
  const float* f16;  // FP16 plans: per-call operand scales (s_b, 1/s_b, s_r, 1/s_r), else null
  const int* gate;   // device stop flag of the solve, or null
  // epilogue
  float* out;
  const float* pmeas;
  void* rq;
  void* rq_lo;
  size_t ps_r;
  int r;
  int tsh;          // 16-bit H^T operand: sample t stored at t + tsh (0 or 4)
  float rq_scale;
  double* partial;
  // residual form only: A c of the current iterate by the momentum recurrence
  // (null: off).  yc [K][Ny][Nx][Nt] holds A c_{k-1} on entry and A c_k on
  // exit, A c_k = (H b + yc_beta A c_{k-1}) yc_inv with yc_inv = 1 / (1 +
  // yc_beta), or H b itself when yc_first; the partial sums are then those of
  // (A c_k - p)^2 instead of r^2
  float* yc;
  float yc_beta, yc_inv;
  int yc_first;
  SwitchParams sw;
  const float* phi;
  const float* stab;
  int nz, nt;
};

__device__ __forceinline__ void block_coords(const BandArgs& A, int& mtile, int& iy, int& ix0,
                                             int& wid) {
  const int nblocks = gridDim.x;
  const int b = blockIdx.x;
  // XCD-aware order: the hardware deals blocks to the 8 XCDs round-robin;
  // give each XCD a contiguous range of the logical tile order so positions
  // that share footprint data run on the same L2.
  const int per = nblocks / 8;
  int lin = b;
  if (b < per * 8) lin = (b % 8) * per + b / 8;
  const int mb = lin % A.n_mblk;
  const int rest = lin / A.n_mblk;
  const int xb = rest % A.nxb;
  iy = rest / A.nxb;
  const int wave = threadIdx.x >> 6;
  mtile = mb * kWavesPerBlock + wave;
  ix0 = xb * kPosPerWave;
  wid = b * kWavesPerBlock + wave;
}

template <int NP>
__device__ __forceinline__ void zero_acc(f32x4 (&acc)[NP]) {
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
}

// Block index with the blocks of each XCD made contiguous: the hardware deals
// blocks to the 8 XCDs round-robin, so block b runs on XCD b % 8; mapping it
// to (b % 8) * (n / 8) + b / 8 gives every XCD one contiguous range of tiles,
// whose neighbours (stencil halos) then come from that XCD's own L2.
__device__ __forceinline__ int xcd_block() {
  const int n = (int)gridDim.x, b = (int)blockIdx.x;
  return (n & 7) == 0 ? (b & 7) * (n >> 3) + (b >> 3) : b;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Epilogue of one 16-pulse block for NP consecutive positions, shared by all
// band kernels (identical accumulator layout: lane l holds output rows
// 4*(l/16)..+3 of column l%16 = pulse kbase + l%16).
//  mode 0: y rows written;  mode 1: r = y - p into the H^T operand, sum r^2
//  into ss;  mode 2: c[s] (+)= sum_k S[k][s] bh[k] (first block writes, later
//  blocks add, always by the same lane, so the order is fixed).
// HALF (a block of at most 8 pulses, staged kernels): accumulator q holds
// the pair of positions 2q, 2q+1, column l%16 = pulse kbase + l%8 of
// position 2q + (l%16)/8; accumulators NP/2.. are unused.
template <int MODE, int NP, int RQ_PREC, bool SPLIT, bool HALF = false>
__device__ __forceinline__ void epi_block(const BandArgs& A, const f32x4 (&acc)[NP], int mtile,
                                          int iy, int ix0, int kbase, bool first, double& ss) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, n = lane & 15;
  const int row0 = mtile * 16 + 4 * g;
  const int k = kbase + (HALF ? (n & 7) : n);
  // accumulator slots and the position of slot p (relative to ix0)
  constexpr int SL = HALF ? NP / 2 : NP;
  const int hsel = HALF ? (n >> 3) : 0;
  auto px = [&](int p) { return HALF ? 2 * p + hsel : p; };
  // undoing the operand's scale: 1/s_b after H, 1/s_r after H^T (FP16 plans
  // take both from the device, chosen per call; the others use inv_scale)
  const float ib = A.f16 ? A.f16[MODE == 2 ? 3 : 1] : A.inv_scale;
  if constexpr (MODE == 0) {
    const int nt = A.nt;
    if (k >= A.nk) return;
#pragma unroll
    for (int p = 0; p < SL; ++p) {
      const int ix = ix0 + px(p);
      if (ix >= A.nx) continue;
      float* yo = A.out + (((size_t)k * A.ny + iy) * A.nx + ix) * nt + row0;
      const f32x4 v = acc[p] * ib;
      if ((nt & 3) == 0 && row0 + 3 < nt) {
        *(f32x4*)yo = v;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (row0 + j < nt) yo[j] = v[j];
      }
    }
  } else if constexpr (MODE == 1 || MODE == 3) {
    constexpr bool REC = MODE == 3;
    const int nt = A.nt;
    if (k >= A.nk) return;
    // 16-bit operand (the staged kernels): the measurements of all NP
    // positions first (one 16-byte load per position where the lane's four
    // samples are aligned and inside the A-scan), so their latency is paid
    // once.  The FP32 kernel has no registers to spare for them (its
    // occupancy would drop) and loads them position by position.
    constexpr bool kPre = RQ_PREC != PSOAM_FP32;
    const bool vec = A.pmeas && ((uintptr_t)A.pmeas & 15) == 0 && (nt & 3) == 0 && row0 + 3 < nt;
    // The operand's row and position strides pass through an empty asm here,
    // so the positions' 64-bit operand addresses are formed per call instead
    // of being hoisted out of the pulse-block loop and held (spilled) across
    // the matrix-core loop
    int xps = A.xp, psr = (int)A.ps_r;
    asm volatile("" : "+s"(xps), "+s"(psr));
    f32x4 pv[kPre ? SL : 1];
    if constexpr (kPre) {
#pragma unroll
      for (int p = 0; p < SL; ++p) {
        const int ix = ix0 + px(p);
        const size_t yi = (((size_t)k * A.ny + iy) * A.nx + ix) * nt + row0;
        if (vec && ix < A.nx) {
          pv[p] = *(const f32x4*)(A.pmeas + yi);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            pv[p][j] = (A.pmeas && ix < A.nx && row0 + j < nt) ? A.pmeas[yi + j] : 0.0f;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < SL; ++p) {
      const int ix = ix0 + px(p);
      if (ix >= A.nx) continue;
      const size_t pos = ((size_t)(iy + A.r) * xps + (ix + A.r)) * (size_t)psr;
      const size_t yi = (((size_t)k * A.ny + iy) * A.nx + ix) * nt + row0;
      float rv[4], pm[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool ok = row0 + j < nt;
        pm[j] = (A.pmeas && ok) ? (kPre ? pv[kPre ? p : 0][j] : A.pmeas[yi + j]) : 0.0f;
        rv[j] = ok ? acc[p][j] * ib - pm[j] : 0.0f;
        if constexpr (!REC) ss += (double)rv[j] * (double)rv[j];
      }
      if constexpr (REC) {
        // A c of the iterate: a convex combination of H b and the stored A c
        // of the previous iterate (same element, same lane: in place)
        float* yp = A.yc + yi;
        const bool v4 = (nt & 3) == 0 && row0 + 3 < nt;
        f32x4 yo = {0.0f, 0.0f, 0.0f, 0.0f};
        if (!A.yc_first) {
          if (v4) {
            yo = *(const f32x4*)yp;
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (row0 + j < nt) yo[j] = yp[j];
          }
        }
        f32x4 yn;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float ya = acc[p][j] * ib;
          yn[j] = A.yc_first ? ya : (ya + A.yc_beta * yo[j]) * A.yc_inv;
        }
        if (v4) {
          *(f32x4*)yp = yn;
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (row0 + j < nt) yp[j] = yn[j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double d = row0 + j < nt ? (double)yn[j] - (double)pm[j] : 0.0;
          ss += d * d;
        }
      }
      if constexpr (RQ_PREC == PSOAM_FP32) {
        float* d = (float*)A.rq + pos + (size_t)row0 * A.kp + k;
#pragma unroll
        for (int j = 0; j < 4; ++j) d[(size_t)j * A.kp] = rv[j];
      } else {
        using H = Half<RQ_PREC>;
        typename H::V4 hi, lo;
        const float rqs = A.f16 ? A.f16[2] : A.rq_scale;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float v = rv[j] * rqs;
          hi[j] = (typename H::E)v;
          lo[j] = (typename H::E)(v - (float)hi[j]);
        }
        // tsh is 0 or 4, so the quarter-octet stays aligned
        const int rs = row0 + A.tsh;
        const size_t o = pos + ((size_t)(rs >> 3) * A.kp + k) * 8 + ((rs >> 2) & 1) * 4;
        *(typename H::V4*)((typename H::E*)A.rq + o) = hi;
        if constexpr (SPLIT) *(typename H::V4*)((typename H::E*)A.rq_lo + o) = lo;
      }
    }
  } else {
    // c[s][iy][ix][z] (+)= sum_k S[k][s] bh[k][z].  The sum over the 16 pulse
    // lanes is a reduce-scatter: each butterfly stage halves the positions a
    // lane keeps, so lane n ends with position n >> (4 - log2 NP) (the low
    // lanes of a pair add once more when NP < 16) and writes its own column.
    static_assert(NP == 8 || NP == 16, "positions per wave");
    static_assert(!HALF || NP == 16, "half blocks: 16 positions per wave");
    constexpr int kSh = NP == 16 ? 0 : 1;
    const int nz = A.nz;
    if (A.sw.diag) {
      // diagonal switching (S_v[k][s] = phi_v if k == s): the lane of pulse k
      // holds species k's column, written directly (pulse blocks cover
      // disjoint species, so no accumulation across calls)
      if (k >= A.nk || k >= A.sw.ns) return;
#pragma unroll
      for (int p = 0; p < SL; ++p) {
        const int ix = ix0 + px(p);
        if (ix >= A.nx) continue;
        const size_t col = ((size_t)iy * A.nx + ix) * nz;
        float* co = A.out + (size_t)k * A.ny * A.nx * nz + col + row0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int z = row0 + j;
          if (z < nz) co[j] = coef_at(A.sw, A.phi, A.stab, A.kp, col, z, k, k) * (acc[p][j] * ib);
        }
      }
      return;
    }
    // the lane's output column after the reduce-scatter
    const int pme = HALF ? 2 * (n & 7) + hsel : n >> kSh;
    const int ixm = ix0 + pme;
    const bool writer = (n & ((1 << kSh) - 1)) == 0 && ixm < A.nx;
    const bool kok = k < A.nk;
    for (int s = 0; s < A.sw.ns; ++s) {
      float x[SL][4];
      if (A.stab) {
        // depth-only switching table: one coefficient per (z, pulse)
        float cz[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int z = row0 + j;
          cz[j] = (kok && z < nz) ? A.stab[((size_t)z * A.kp + k) * A.sw.ns + s] * ib : 0.0f;
        }
#pragma unroll
        for (int p = 0; p < SL; ++p)
#pragma unroll
          for (int j = 0; j < 4; ++j) x[p][j] = cz[j] * acc[p][j];
      } else {
#pragma unroll
        for (int p = 0; p < SL; ++p) {
          const int ix = ix0 + px(p);
          const int ixc = ix < A.nx ? ix : A.nx - 1;
          const size_t col = ((size_t)iy * A.nx + ixc) * nz;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int z = row0 + j;
            x[p][j] = (kok && z < nz) ? scoef(A.sw, A.phi[col + z], k, s) * (acc[p][j] * ib) : 0.0f;
          }
        }
      }
      // reduce-scatter over lane bits 3, 2, ... (half blocks: 2, 1, 0; bit 3
      // tells the two positions of a pair apart): the upper half of the
      // lanes keeps the upper half of the slots
#pragma unroll
      for (int h = SL / 2, mask = HALF ? 4 : 8; h >= 1; h >>= 1, mask >>= 1) {
        const bool up = (n & mask) != 0;
#pragma unroll
        for (int q = 0; q < h; ++q)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float send = up ? x[q][j] : x[q + h][j];
            const float keep = up ? x[q + h][j] : x[q][j];
            x[q][j] = keep + __shfl_xor(send, mask, 64);
          }
      }
      if constexpr (kSh == 1) {
#pragma unroll
        for (int j = 0; j < 4; ++j) x[0][j] += __shfl_xor(x[0][j], 1, 64);
      }
      if (writer) {
        float* co = A.out + ((size_t)s * A.ny * A.nx + (size_t)iy * A.nx + ixm) * nz + row0;
        if ((nz & 3) == 0 && row0 + 3 < nz) {
          f32x4 v = {x[0][0], x[0][1], x[0][2], x[0][3]};
          if (!first) v += *(const f32x4*)co;
          *(f32x4*)co = v;
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (row0 + j < nz) co[j] = first ? x[0][j] : co[j] + x[0][j];
        }
      }
    }
  }
}

// Band kernel reading its operand straight from global memory: one wave owns
// one output tile x kPosPerWave positions x all pulse blocks.  Used when the
// staged variant below does not fit in LDS, and for FP32.
template <int PREC, bool SPLIT, int NB, int MODE>
__global__ __launch_bounds__(256) void band16(BandArgs A) {
  if (A.gate && *A.gate) return;  // a device stop test has ended the solve
  using H = Half<PREC>;
  using E = typename H::E;
  using V = typename H::V;
  int mtile, iy, ix0, wid;
  block_coords(A, mtile, iy, ix0, wid);
  const int lane = threadIdx.x & 63;
  if (mtile >= A.n_mtiles) {
    if ((MODE == 1 || MODE == 3) && lane == 0) A.partial[wid] = 0.0;
    return;
  }
  const int g = lane >> 4, n = lane & 15;
  f32x4 acc[NB][kPosPerWave];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) zero_acc(acc[nb]);
  const int c0 = A.start[mtile], c1 = A.start[mtile + 1];
  const size_t base = ((size_t)iy * A.xp + ix0) * A.ps + (size_t)n * 8;
  const E* q = (const E*)A.q + base;
  const E* qlo = SPLIT ? (const E*)A.q_lo + base : nullptr;
  const V* av = (const V*)A.a;
  const V* avlo = (const V*)A.a_lo;
  for (int c = c0; c < c1; ++c) {
    const int off = A.off[c * 4 + g];
    const V a = av[(size_t)c * kWaveLanes + lane];
    V alo{};
    if constexpr (SPLIT) alo = avlo[(size_t)c * kWaveLanes + lane];
    const E* qc = q + off;
#pragma unroll
    for (int p = 0; p < kPosPerWave; ++p) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const V b = *(const V*)(qc + p * A.ps + nb * 128);
        acc[nb][p] = H::mma(a, b, acc[nb][p]);
        if constexpr (SPLIT) {
          const V blo = *(const V*)(qlo + off + p * A.ps + nb * 128);
          acc[nb][p] = H::mma(a, blo, acc[nb][p]);
          acc[nb][p] = H::mma(alo, b, acc[nb][p]);
        }
      }
    }
  }
  double ss = 0.0;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
    epi_block<MODE, kPosPerWave, PREC, SPLIT>(A, acc[nb], mtile, iy, ix0, nb * 16, nb == 0, ss);
  if constexpr (MODE == 1 || MODE == 3) {
    ss = wave_sum(ss);
    if (lane == 0) A.partial[wid] = ss;
  }
}

template <int NB, int MODE>
__global__ __launch_bounds__(256) void band32(BandArgs A) {
  if (A.gate && *A.gate) return;  // a device stop test has ended the solve
  int mtile, iy, ix0, wid;
  block_coords(A, mtile, iy, ix0, wid);
  const int lane = threadIdx.x & 63;
  if (mtile >= A.n_mtiles) {
    if ((MODE == 1 || MODE == 3) && lane == 0) A.partial[wid] = 0.0;
    return;
  }
  const int g = lane >> 4, n = lane & 15;
  f32x4 acc[NB][kPosPerWave];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) zero_acc(acc[nb]);
  const int c0 = A.start[mtile], c1 = A.start[mtile + 1];
  const float* q = (const float*)A.q + ((size_t)iy * A.xp + ix0) * A.ps + n;
  const float* av = (const float*)A.a;
  for (int c = c0; c < c1; ++c) {
    const int off = A.off[c * 4 + g];
    const float a = av[(size_t)c * kWaveLanes + lane];
    const float* qc = q + off;
#pragma unroll
    for (int p = 0; p < kPosPerWave; ++p) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float b = qc[p * A.ps + nb * 16];
        acc[nb][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[nb][p], 0, 0, 0);
      }
    }
  }
  double ss = 0.0;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
    epi_block<MODE, kPosPerWave, PSOAM_FP32, false>(A, acc[nb], mtile, iy, ix0, nb * 16, nb == 0,
                                                    ss);
  if constexpr (MODE == 1 || MODE == 3) {
    ss = wave_sum(ss);
    if (lane == 0) A.partial[wid] = ss;
  }
}

// --------------------------------------------------------------------------
// LDS-staged band kernel (16-bit operands).
//
// A workgroup owns ROWS (4 or 8) consecutive output rows (one per wave) x
// kLdsPos consecutive positions x one output tile of 16 rows.  Input rows
// are streamed through LDS: padded input row iy0 + j is staged once (only the
// octets the tile needs for the dy values j - r of its waves, one 16-pulse
// block at a time) and every wave whose dy = j - wave is in the footprint
// contracts against it.  The band blocks come from a chunk list per
// (tile, dy); each group names (octet, dx), so the operand of position p is
// the staged column p + dx.
// --------------------------------------------------------------------------

struct LdsArgs {
  const int* lstart;       // [n_mtiles * F + 1]
  const uint32_t* lgrp;    // [chunks * 4]: octet << 16 | dx  (octet 0xffff = padding group)
  const uint32_t* win;     // [n_mtiles * (F + ROWS - 1)]: obase << 16 | ocnt
  const void* la;
  const void* la_lo;
  int f, yp, nyb, nxb, lds_elems;
  int meta_off;  // byte offset of the per-tile window / run tables in LDS
  const int* order;  // output tiles by decreasing work
  const int* rinfo;  // [runs][2]: length, first chunk
  int max_runs;      // most runs of one tile
  int la_bytes;      // bytes of la (and la_lo), including kRunMax zero chunks at the end
};

// LOADW > 0 (one-part operands, one workgroup per CU): LOADW loader waves
// beside the ROWS contracting waves.  The loaders hold the next staged row in
// registers (up to kLoadItems 16-byte items per thread) while the other waves
// contract the current one, and write it to LDS between two barriers, so the
// row's load latency is hidden behind the matrix cores instead of stalling
// every wave of the workgroup; the loads sit on the loaders' own memory
// counters, so the contracting waves' waits for band blocks never wait for
// them.  kLoadItems * 64 * LOADW must cover the widest window (plan time).
constexpr int kLoadItems = 25;
template <int PREC, bool SPLIT, int MODE, int ROWS, int LOADW>
__device__ __forceinline__ void band16_lds_body(const BandArgs& A, const LdsArgs& L) {
  static_assert(LOADW == 0 || !SPLIT, "loader waves stage one-part operands");
  if (A.gate && *A.gate) return;  // a device stop test has ended the solve
  using H = Half<PREC>;
  using E = typename H::E;
  using V = typename H::V;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  E* sh = (E*)smem_raw;
  // per-tile row windows, run bounds and run records, read once into LDS
  uint32_t* s_win = (uint32_t*)(smem_raw + L.meta_off);
  int* s_lstart = (int*)(s_win + (L.f + ROWS - 1));
  uint32_t* s_rgrp = (uint32_t*)(s_lstart + L.f + 1);      // [max_runs][4]
  int* s_rinfo = (int*)(s_rgrp + 4 * L.max_runs);           // [max_runs][2]
  // Block order.  Output tiles differ several-fold in work (bands crowd
  // around the focal time), so (1) every XCD (blocks are dealt to the 8 XCDs
  // round-robin) receives all tiles for its own share of position blocks,
  // and (2) within an XCD the heaviest tiles are dispatched first so the
  // light ones fill the tail (longest-processing-time order, L.order).
  // When the position blocks do not divide by 8, each XCD's share is rounded
  // up and the blocks past the last position have no work (the grid holds
  // 8 ceil(npos / 8) blocks per tile).
  const int b = blockIdx.x;
  const int npos = L.nxb * L.nyb;
  const int per_x = (npos + 7) >> 3;
  const int xcd = b & 7, kx = b >> 3;
  const int mtile = L.order[kx / per_x];
  const int pos = xcd * per_x + kx % per_x;
  constexpr int NTALL = 64 * (ROWS + LOADW);             // threads of the workgroup
  constexpr int NT = 64 * (LOADW > 0 ? LOADW : ROWS);    // threads that stage rows
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  if (pos >= npos) {
    // no positions: the residual form still owns its partial sums
    if constexpr (MODE == 1 || MODE == 3)
      if (lane == 0 && wave < ROWS) A.partial[(size_t)b * ROWS + wave] = 0.0;
    return;
  }
  const int xb = pos % L.nxb;
  const int yb = pos / L.nxb;
  const int g = lane >> 4, n = lane & 15;
  const int iy0 = yb * ROWS, ix0 = xb * kLdsPos;
  const int iy = iy0 + wave;
  const bool loader = LOADW > 0 && wave >= ROWS;          // uniform per wave
  const bool row_ok = !loader && iy < A.ny;
  // this thread's index among the staging threads
  const int st_id = (int)threadIdx.x - (LOADW > 0 ? 64 * ROWS : 0);
  const int F = L.f;
  const int XW = kLdsPos + F - 1;
  const int nwin = F + ROWS - 1;
  const V* av = (const V*)L.la;
  const V* avlo = (const V*)L.la_lo;
  const E* q = (const E*)A.q;
  const E* qlo = (const E*)A.q_lo;
  {
    const int nw = L.f + ROWS - 1;
    for (int i = (int)threadIdx.x; i < nw; i += NTALL) s_win[i] = L.win[mtile * nw + i];
    const int rt0 = L.lstart[mtile * L.f];
    for (int i = (int)threadIdx.x; i <= L.f; i += NTALL) s_lstart[i] = L.lstart[mtile * L.f + i] - rt0;
    const int nrun = L.lstart[(mtile + 1) * L.f] - rt0;
    for (int i = (int)threadIdx.x; i < 4 * nrun; i += NTALL) s_rgrp[i] = L.lgrp[4 * rt0 + i];
    for (int i = (int)threadIdx.x; i < 2 * nrun; i += NTALL) s_rinfo[i] = L.rinfo[2 * rt0 + i];
    __syncthreads();
  }
  double ss = 0.0;
  const int nb_n = A.kp / 16;
  // Half form of the last block (at most 8 pulses in it): 8 pulses per staged
  // column, and the matrix cores' 16 columns take 8 pulses of two positions
  auto half_pb = [&](int pb_r) { return A.half != 0 && pb_r == nb_n - 1; };
  // Band blocks of the current run, in registers.  Each run loads the next
  // run's blocks slot by slot as its own chunks finish with them, so the
  // loads are in flight while the remaining chunks compute.
  // Slot i of a run holds chunk (first chunk + i); slots past the run's
  // length read the following chunks (or the zero chunks that end the table)
  // and are not used.  Buffer loads share one offset register per run.
  const int nrun = L.lstart[(mtile + 1) * L.f] - L.lstart[mtile * L.f];
  const __amdgpu_buffer_rsrc_t rs_hi = __builtin_amdgcn_make_buffer_rsrc((void*)L.la, (short)0, L.la_bytes, kBufWord3);
  const __amdgpu_buffer_rsrc_t rs_lo =
      __builtin_amdgcn_make_buffer_rsrc((void*)(SPLIT ? L.la_lo : L.la), (short)0, L.la_bytes, kBufWord3);
  // cb is wave-uniform: the lane offset is the only vector address operand
  const int vo = lane * (int)sizeof(V);
  auto load_run = [&](int cb, V (&ab)[kRunMax], V (&al)[SPLIT ? kRunMax : 1], int i) {
    const int so = (cb + i) * kWaveLanes * (int)sizeof(V);
    ab[i] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(rs_hi, vo, so, 0));
    if constexpr (SPLIT) al[i] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(rs_lo, vo, so, 0));
  };
  V ab[kRunMax];
  V al[SPLIT ? kRunMax : 1];
  if (row_ok && nrun > 0) {
    const int cb0 = __builtin_amdgcn_readfirstlane(s_rinfo[1]);
#pragma unroll
    for (int i = 0; i < kRunMax; ++i) load_run(cb0, ab, al, i);
  }
  __builtin_amdgcn_s_waitcnt(kVmcnt0);
  // Staging: thread t loads items t, t+NT, ... of the row, where item
  // it = (oi*XW + xi)*16 + nn is one 16-byte octet of pulse nn at column xi
  // of octet oi; nn = t%16 is fixed and (xi, oi) advance by NT/16 columns
  // per step (half blocks: 8 pulses per column, it = (oi*XW + xi)*8 + nn,
  // nn = t%8, NT/8 columns per step).  Without loader waves every thread
  // stages, with buffer loads that write LDS directly.  The split forms stage
  // the high and the low operand rows in two passes over the window (the
  // same LDS tile): pass 0 adds hi(H) hi(q) + lo(H) hi(q), pass 1 adds
  // hi(H) lo(q).
  const int ps = (int)A.ps;
  const int row_bytes = A.xp * ps * (int)sizeof(E);
  const int dwrap = -XW * ps + A.kp * 8;
  // A thread's walk over items u0*NT + t, (u0+1)*NT + t, ... of staged row
  // jr of pulse block pb_r: the row's buffer, and per item its column xi and
  // element offset off.  A step of cpt columns is qw whole octet windows and
  // rw more columns, then at most one wrap into the next octet (selects, no
  // branches).
  struct Walk {
    int xi, off, rw, dstep;
  };
  auto walk_start = [&](int u0, int jr, int pb_r, int pass_r, __amdgpu_buffer_rsrc_t& rq) {
    const bool hf = half_pb(pb_r);
    const int cpt = hf ? NT / 8 : NT / 16;  // columns per step
    const int obase_r = (int)(s_win[jr] >> 16);
    rq = __builtin_amdgcn_make_buffer_rsrc(
        (void*)((pass_r ? qlo : q) + (size_t)(iy0 + jr) * A.xp * A.ps), (short)0, row_bytes, kBufWord3);
    const int r2 = u0 * cpt + (hf ? st_id >> 3 : st_id >> 4);
    const int qw = cpt / XW;
    Walk w;
    w.xi = r2 % XW;
    w.off = (ix0 + w.xi) * ps + ((obase_r + r2 / XW) * A.kp + pb_r * 16 + (st_id & (hf ? 7 : 15))) * 8;
    w.rw = cpt - qw * XW;
    w.dstep = w.rw * ps + qw * A.kp * 8;
    return w;
  };
  auto walk_next = [&](Walk& w) {
    w.xi += w.rw;
    w.off += w.dstep;
    const bool w1 = w.xi >= XW;
    w.xi = w1 ? w.xi - XW : w.xi;
    w.off = w1 ? w.off + dwrap : w.off;
  };
  // loader waves: cnt items into registers (all loads unconditional: an item
  // past the window still lies inside the padded row, and its value is never
  // written to LDS)
  auto issue = [&](V* tmp, int cnt, int u0, int jr, int pb_r, int pass_r) {
    __amdgpu_buffer_rsrc_t rq;
    Walk w = walk_start(u0, jr, pb_r, pass_r, rq);
#pragma unroll
    for (int u = 0; u < cnt; ++u) {
      tmp[u] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(rq, w.off * (int)sizeof(E), 0, 0));
      walk_next(w);
    }
  };
  // a staged row is skipped when its window is empty or it lies past the
  // padded grid (uniform over the block)
  auto staged = [&](int jr) { return (s_win[jr] & 0xffffu) != 0 && iy0 + jr < L.yp; };
  auto row_from = [&](int jr) {
    for (int k2 = jr; k2 < nwin; ++k2)
      if (staged(k2)) return k2;
    return nwin;
  };
  if constexpr (LOADW > 0) {
    if (loader) {
      // The loader waves' own loop: the same staged rows, the same two
      // barriers per row as the contracting waves' loop below.  A row is
      // written to LDS between the barriers; the next row (or the next pulse
      // block's first) is then loaded while the other waves contract.
      V pf[kLoadItems];
      {
        const int j0 = row_from(0);
        if (j0 < nwin) issue(pf, kLoadItems, 0, j0, 0, 0);
      }
      for (int pb = 0; pb < nb_n; ++pb)
        for (int j = 0; j < nwin; ++j) {
          if (!staged(j)) continue;
          __syncthreads();  // the previous row's contractions are done with LDS
          const int items = (int)(s_win[j] & 0xffffu) * XW * (half_pb(pb) ? 8 : 16);
          __builtin_amdgcn_s_waitcnt(kVmcnt0);  // row j has arrived
#pragma unroll
          for (int u = 0; u < kLoadItems; ++u) {
            const int it = u * NT + st_id;
            if (it < items) *(V*)(sh + it * 8) = pf[u];
          }
          __syncthreads();
          // next in staging order: a later row of this block, else the next
          // block's first row
          int jn = row_from(j + 1), pbn = pb;
          if (jn == nwin) {
            jn = row_from(0);
            pbn = pb + 1;
          }
          if (jn < nwin && pbn < nb_n) issue(pf, kLoadItems, 0, jn, pbn, 0);
        }
      return;
    }
  }
  for (int pb = 0; pb < nb_n; ++pb) {
    const bool hf = half_pb(pb);
    f32x4 acc[kLdsPos];
    zero_acc(acc);
    for (int pass = 0; pass < (SPLIT ? 2 : 1); ++pass)
    for (int j = 0; j < nwin; ++j) {
      const uint32_t wj = s_win[j];
      const int ocnt = (int)(wj & 0xffffu), obase = (int)(wj >> 16);
      if (!staged(j)) continue;
      __syncthreads();  // the previous row's contractions are done with LDS
      if constexpr (LOADW == 0) {
        // Every item of the row goes straight from global memory to LDS
        // (buffer loads with the LDS destination: no registers, no LDS write
        // instructions), all of a thread's items in flight at once.  A wave's
        // 64 lanes fill 64 consecutive 16-byte slots, so item u*NT + t lands
        // at slot u*NT + t as the LDS layout wants; lanes past the window
        // are masked off and write nothing.
        const int items = ocnt * XW * (hf ? 8 : 16);
        __amdgpu_buffer_rsrc_t rq;
        Walk w = walk_start(0, j, pb, pass, rq);
        const int wbase = __builtin_amdgcn_readfirstlane((int)threadIdx.x & ~63);
        for (int u = 0; u * NT < items; ++u) {
          if (u * NT + st_id < items)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rq, (__attribute__((address_space(3))) void*)(sh + (u * NT + wbase) * 8), 16,
                w.off * (int)sizeof(E), 0, 0, 0);
          walk_next(w);
        }
        __builtin_amdgcn_s_waitcnt(kVmcnt0);  // this thread's items are in LDS
      }
      __syncthreads();  // row j is in LDS
      const int dy = j - wave;
      if (row_ok && dy >= 0 && dy < F && hf) {
        // Half block: the staged column holds 8 pulses, and the fragment of
        // slot q is the two columns of positions 2q, 2q+1 (lanes 0-7, 8-15).
        // Stepping dx by -1 moves a pair by one column, i.e. by half a pair,
        // so the window keeps the 15 overlapping pairs that start at offsets
        // 0..14 from the run's first column (one LDS read each) and adds the
        // pair starting at -i at chunk i; slot q at chunk i is the pair at
        // offset 2q - i (index mod 16: an overwritten pair is never needed
        // again).
        const int r0 = __builtin_amdgcn_readfirstlane(s_lstart[dy]);
        const int r1 = __builtin_amdgcn_readfirstlane(s_lstart[dy + 1]);
        for (int rr = r0; rr < r1; ++rr) {
          const uint32_t gr = s_rgrp[4 * rr + g];
          const int m = __builtin_amdgcn_readfirstlane(s_rinfo[2 * rr]);
          const int d = (int)(gr & 0xffffu);
          const int oo = (int)(gr >> 16) - obase;
          const int base = ((oo * XW + d) * 8 + n) * 8;
          const int nx = rr + 1 == nrun ? 0 : rr + 1;
          const int cb2 = __builtin_amdgcn_readfirstlane(s_rinfo[2 * nx + 1]);
          V R[16];
#pragma unroll
          for (int o = 0; o < 15; ++o) R[o] = *(const V*)(sh + base + o * 64);
#pragma unroll
          for (int i = 0; i < kRunMax; ++i) {
            if (i < m) {
              if (i > 0) R[(16 - i) & 15] = *(const V*)(sh + base - i * 64);
              // slot 0 takes the pair just read, so it goes last
              if (SPLIT && pass == 0) {
#pragma unroll
                for (int t = 1; t <= 8; ++t) {
                  const int qs = t & 7;
                  const int w = (2 * qs - i) & 15;
                  acc[qs] = H::mma(ab[i], R[w], acc[qs]);
                  acc[qs] = H::mma(al[i], R[w], acc[qs]);
                }
              } else {
#pragma unroll
                for (int t = 1; t <= 8; ++t) {
                  const int qs = t & 7;
                  acc[qs] = H::mma(ab[i], R[(2 * qs - i) & 15], acc[qs]);
                }
              }
            }
            load_run(cb2, ab, al, i);
          }
        }
      } else if (row_ok && dy >= 0 && dy < F) {
        // Runs of this (tile, dy).  Within a run the four groups keep their
        // octet and step their offset by -1 per chunk, so position p's operand
        // at chunk i is position p-1's at chunk i-1: a 16-fragment register
        // window slides and one new column is read from LDS per chunk.
        const int r0 = __builtin_amdgcn_readfirstlane(s_lstart[dy]);
        const int r1 = __builtin_amdgcn_readfirstlane(s_lstart[dy + 1]);
        for (int rr = r0; rr < r1; ++rr) {
          const uint32_t gr = s_rgrp[4 * rr + g];
          const int m = __builtin_amdgcn_readfirstlane(s_rinfo[2 * rr]);
          const int d = (int)(gr & 0xffffu);
          const int oo = (int)(gr >> 16) - obase;
          const int base = ((oo * XW + d) * 16 + n) * 8;
          // the run after this one (the first of the tile after the last: the
          // band blocks do not depend on the pulse block)
          const int nx = rr + 1 == nrun ? 0 : rr + 1;
          const int cb2 = __builtin_amdgcn_readfirstlane(s_rinfo[2 * nx + 1]);
          V R[kLdsPos];
#pragma unroll
          for (int p = 0; p < kLdsPos; ++p) R[p] = *(const V*)(sh + base + p * 128);
#pragma unroll
          for (int i = 0; i < kRunMax; ++i) {
            if (i < m) {
              if (i > 0) R[(kLdsPos - i) & (kLdsPos - 1)] = *(const V*)(sh + base - i * 128);
              // position 0 takes the column just read from LDS, so it goes
              // last: the other fifteen products cover the read's latency
              if (SPLIT && pass == 0) {
#pragma unroll
                for (int q = 1; q <= kLdsPos; ++q) {
                  const int p = q & (kLdsPos - 1);
                  const int w = (p - i) & (kLdsPos - 1);
                  acc[p] = H::mma(ab[i], R[w], acc[p]);
                  acc[p] = H::mma(al[i], R[w], acc[p]);
                }
              } else {
#pragma unroll
                for (int q = 1; q <= kLdsPos; ++q) {
                  const int p = q & (kLdsPos - 1);
                  acc[p] = H::mma(ab[i], R[(p - i) & (kLdsPos - 1)], acc[p]);
                }
              }
            }
            // slot i is free: load the next run's block i into it
            load_run(cb2, ab, al, i);
          }
        }
      }
    }
    if (row_ok) {
      if (hf)
        epi_block<MODE, kLdsPos, PREC, SPLIT, true>(A, acc, mtile, iy, ix0, pb * 16, pb == 0, ss);
      else
        epi_block<MODE, kLdsPos, PREC, SPLIT>(A, acc, mtile, iy, ix0, pb * 16, pb == 0, ss);
    }
    // Retire the epilogue's stores here: with stores and loads both in
    // flight the memory counter no longer orders the band-block loads, and
    // every chunk of the run loop would wait for all of them.
    __builtin_amdgcn_s_waitcnt(kVmcnt0);
  }
  if constexpr (MODE == 1 || MODE == 3) {
    ss = wave_sum(ss);
    if (lane == 0 && !loader) A.partial[(size_t)b * ROWS + wave] = ss;
  }
}

// --------------------------------------------------------------------------
// FP32 band contraction over the run-packed table (single-sample groups).
//
// The staged kernel's runs without the staging: a wave owns one output row x
// kLdsPos positions x one output tile, walks every dy of the footprint and
// every run of (tile, dy), and keeps a 16-fragment register window of the
// operand (one float per lane: sample l of its group, pulse n) that slides
// one column per chunk, so a chunk reads one new column from global memory
// (the neighbouring waves and positions read the same rows: L1/L2 hits) and
// issues kLdsPos products.  The band values (one float per lane per chunk)
// are loaded a run ahead into a ring of kRunMax slots, as in the staged
// kernel.  A block holds kWavesPerBlock consecutive output rows; blocks are
// ordered by XCD and tile work like the staged kernel's.
// --------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(64 * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(MODE == 2 ? 2 : 3))) void band32_run(
    BandArgs A, LdsArgs L) {
  if (A.gate && *A.gate) return;  // a device stop test has ended the solve
  const int b = blockIdx.x;
  const int npos = L.nxb * L.nyb;
  int mtile, pos;
  if ((npos & 7) == 0) {
    const int xcd = b & 7, k = b >> 3;
    const int per_x = npos >> 3;
    mtile = L.order[k / per_x];
    pos = xcd * per_x + k % per_x;
  } else {
    mtile = L.order[b / npos];
    pos = b % npos;
  }
  const int xb = pos % L.nxb, yb = pos / L.nxb;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, n = lane & 15;
  const int iy = yb * kWavesPerBlock + wave, ix0 = xb * kLdsPos;
  const int F = L.f;
  double ss = 0.0;
  if (iy < A.ny) {
    const int rt0 = L.lstart[mtile * F];
    const int rt1 = L.lstart[(mtile + 1) * F];
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)L.la, (short)0, L.la_bytes, kBufWord3);
    const int vo = lane * (int)sizeof(float);
    float ab[kRunMax];
    auto load_run = [&](int cb, int i) {
      ab[i] = __builtin_bit_cast(
          float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, (cb + i) * kWaveLanes * (int)sizeof(float), 0));
    };
    const float* q = (const float*)A.q;
    const int nb_n = A.kp / 16;
    for (int pb = 0; pb < nb_n; ++pb) {
      f32x4 acc[kLdsPos];
      zero_acc(acc);
      if (pb == 0 && rt1 > rt0) {
        const int cb0 = __builtin_amdgcn_readfirstlane(L.rinfo[2 * rt0 + 1]);
#pragma unroll
        for (int i = 0; i < kRunMax; ++i) load_run(cb0, i);
      }
      for (int dy = 0; dy < F; ++dy) {
        const int r0 = __builtin_amdgcn_readfirstlane(L.lstart[mtile * F + dy]);
        const int r1 = __builtin_amdgcn_readfirstlane(L.lstart[mtile * F + dy + 1]);
        // padded input row iy + dy; column ix0 + x of the padded grid
        const float* qrow = q + (size_t)(iy + dy) * A.xp * A.ps + (size_t)ix0 * A.ps + pb * 16 + n;
        for (int rr = r0; rr < r1; ++rr) {
          const uint32_t gr = L.lgrp[4 * rr + g];
          const int m = __builtin_amdgcn_readfirstlane(L.rinfo[2 * rr]);
          const int d = (int)(gr & 0xffffu);
          const int l = (int)(gr >> 16);
          const float* base = qrow + (size_t)d * A.ps + (size_t)l * A.kp;
          // the run after this one (the first of the tile after the last)
          const int nx = rr + 1 == rt1 ? rt0 : rr + 1;
          const int cb2 = __builtin_amdgcn_readfirstlane(L.rinfo[2 * nx + 1]);
          float R[kLdsPos];
#pragma unroll
          for (int p = 0; p < kLdsPos; ++p) R[p] = base[(size_t)p * A.ps];
#pragma unroll
          for (int i = 0; i < kRunMax; ++i) {
            if (i < m) {
              if (i > 0) R[(kLdsPos - i) & (kLdsPos - 1)] = base[-(ptrdiff_t)i * A.ps];
#pragma unroll
              for (int t = 1; t <= kLdsPos; ++t) {
                const int p = t & (kLdsPos - 1);
                acc[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(ab[i], R[(p - i) & (kLdsPos - 1)],
                                                                acc[p], 0, 0, 0);
              }
            }
            load_run(cb2, i);
          }
        }
      }
      epi_block<MODE, kLdsPos, PSOAM_FP32, false>(A, acc, mtile, iy, ix0, pb * 16, pb == 0, ss);
    }
  }
  if constexpr (MODE == 1 || MODE == 3) {
    ss = wave_sum(ss);
    if (lane == 0) A.partial[(size_t)b * kWavesPerBlock + wave] = ss;
  }
}

// H and the residual form are held to three waves per SIMD where three can
// share it: 4-row workgroups with one-part operands (three of ~47 KB share a
// CU at 31 x 31 footprints) and 8-row ones with loader waves (twelve waves).
// An 8-row workgroup without loader waves runs two waves per SIMD whatever
// its registers (a second one would need four), and split operands need the
// registers for their second band-block buffer: these get 256.  A 12-row
// workgroup (one-part operands) needs three waves per SIMD resident.
template <int PREC, bool SPLIT, int MODE, int ROWS, int LOADW>
__global__ __launch_bounds__(64 * (ROWS + LOADW)) __attribute__((amdgpu_waves_per_eu((SPLIT || (ROWS == 8 && LOADW == 0)) ? 2 : 3))) void band16_lds(
    BandArgs A, LdsArgs L) {
  band16_lds_body<PREC, SPLIT, MODE, ROWS, LOADW>(A, L);
}

// H^T with one-part operands is held to two waves per SIMD (256 registers)
// so that two 4-row workgroups can share a CU when their staged window fits;
// a 12-row workgroup needs three
template <int PREC, bool SPLIT, int ROWS, int LOADW>
__global__ __launch_bounds__(64 * (ROWS + LOADW)) __attribute__((amdgpu_waves_per_eu(SPLIT ? 1 : (ROWS == 12 ? 3 : 2)))) void band16_lds_adj(
    BandArgs A, LdsArgs L) {
  band16_lds_body<PREC, SPLIT, 2, ROWS, LOADW>(A, L);
}

// the calling thread's device stop gate (see set_gate)
static thread_local const int* t_gate = nullptr;
void set_gate(const int* g) { t_gate = g; }
const int* gate_now() { return t_gate; }

// --------------------------------------------------------------------------
// FP16 operand scales.  Every FP16 operand is written times a power of two
// chosen on the device right before, from an FP32 max-abs reduction of what
// is converted (or a bound that holds for every element of it), so that the
// largest value lands at or below 2^14: nothing overflows FP16's 65504 and
// the precision of every value down to 2^-28 of the largest is the format's.
// A power-of-two scale is exact, so results do not depend on it except where
// a fixed scale would have overflowed or left the normal range.
// --------------------------------------------------------------------------

// running max |x| into acc (float bits: nonnegative floats order as unsigned
// integers); NaN inputs are skipped, an infinite one gives scale 1
__global__ __launch_bounds__(256) void f16_amax_kernel(const float* __restrict__ x, int64_t n,
                                                       unsigned* acc,
                                                       const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  __shared__ float sm[4];
  float m = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    m = fmaxf(m, fabsf(x[i]));
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(sm[0], sm[1]), fmaxf(sm[2], sm[3]));
    atomicMax(acc, __float_as_uint(m));
  }
}

// one thread: mode 0 sets s_b from acc[0] * c1 (and keeps the max as st[4]);
// mode 1 sets s_r from acc[1] * c1; mode 2 keeps acc[1] as max |p| (st[5]);
// mode 3 sets s_r from the bound c1 st[4] + c2 st[5].  The accumulator read
// is cleared for its next use.
__global__ void f16_scale_kernel(float* st, unsigned* acc, int mode, float c1, float c2,
                                 const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  auto pow2 = [](float bound) {
    if (!(bound > 0.0f) || !isfinite(bound)) return 1.0f;
    int e = 14 - (int)ceilf(log2f(bound));
    e = e < -100 ? -100 : (e > 100 ? 100 : e);
    return ldexpf(1.0f, e);
  };
  float sc = 1.0f;
  int slot = 2;
  if (mode == 0) {
    const float a = __uint_as_float(acc[0]);
    acc[0] = 0u;
    st[4] = a;
    sc = pow2(a * c1);
    slot = 0;
  } else if (mode == 1) {
    const float a = __uint_as_float(acc[1]);
    acc[1] = 0u;
    sc = pow2(a * c1);
  } else if (mode == 2) {
    st[5] = __uint_as_float(acc[1]);
    acc[1] = 0u;
    return;
  } else {
    sc = pow2(c1 * st[4] + c2 * st[5]);
  }
  st[slot] = sc;
  st[slot + 1] = 1.0f / sc;
}

static hipError_t f16_amax(const psoam_plan* P, const float* x, int64_t n, int slot,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t want = (n + 255) / 256;
  const unsigned nb = (unsigned)std::min<int64_t>(want, 2048);
  hipLaunchKernelGGL(f16_amax_kernel, dim3(nb), dim3(256), 0, s, x, n, P->d_f16acc + slot,
                     gate_now());
  return hipGetLastError();
}

static hipError_t f16_scale(const psoam_plan* P, int mode, double c1, double c2, hipStream_t s) {
  hipLaunchKernelGGL(f16_scale_kernel, dim3(1), dim3(1), 0, s, P->d_f16, P->d_f16acc, mode,
                     (float)c1, (float)c2, gate_now());
  return hipGetLastError();
}

hipError_t launch_f16_pmax(const psoam_plan* P, const float* p, hipStream_t s) {
  if (!P->d_f16) return hipSuccess;
  if (p) {
    const hipError_t e = f16_amax(P, p, (int64_t)P->y_elems(), 1, s);
    if (e != hipSuccess) return e;
  }
  return f16_scale(P, 2, 0.0, 0.0, s);
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
static inline unsigned blocks_for(size_t n, unsigned bs = 256) {
  return (unsigned)((n + bs - 1) / bs);
}

hipError_t launch_switch_fwd(const psoam_plan* P, const float* c, hipStream_t s) {
  const auto& g = P->g;
  const float* stab = P->d_stab;
  if (P->d_f16) {
    // |b_k| <= sum_s |S_v[k][s]| |c_s| <= srow max |c|
    hipError_t e = f16_amax(P, c, (int64_t)P->c_elems(), 0, s);
    if (e == hipSuccess) e = f16_scale(P, 0, P->srow, 0.0, s);
    if (e != hipSuccess) return e;
  }
  const int vec = P->d_stab_o && (g.nz % 8) == 0 && ((uintptr_t)c & 15) == 0;
  switch (P->prec) {
    case PSOAM_FP32: {
      const size_t n = (size_t)g.ny * g.nx * g.nz * P->Kp;
      hipLaunchKernelGGL(switch_fwd32, dim3(blocks_for(n)), dim3(256), 0, s, c, P->d_phi, stab,
                         P->sw, (float*)P->d_bq, g.ny, g.nx, g.nz, P->Kp, P->Xp, P->R, P->ps_b,
                         gate_now());
      break;
    }
#define PSOAM_SW16(PR, SP)                                                                  \
  {                                                                                         \
    using E = Half<PR>::E;                                                                  \
    const size_t n = (size_t)g.ny * g.nx * (P->Lz / 8) * P->Kp;                            \
    hipLaunchKernelGGL((switch_fwd16<PR, SP>), dim3(blocks_for(n)), dim3(256), 0, s, c,     \
                       P->d_phi, stab, P->d_stab_o, vec, P->d_f16, P->sw, (E*)P->d_bq,     \
                       (E*)P->d_bq_lo, g.ny, g.nx, g.nz, P->Lz / 8, P->Kp, P->Xp, P->R,    \
                       P->ps_b, gate_now());                                                \
    break;                                                                                  \
  }
    case PSOAM_BF16:
    case PSOAM_BF16_REFINED: PSOAM_SW16(PSOAM_BF16, false)
    case PSOAM_FP16: PSOAM_SW16(PSOAM_FP16, false)
    case PSOAM_BF16_SPLIT: PSOAM_SW16(PSOAM_BF16, true)
    case PSOAM_FP16_SPLIT: PSOAM_SW16(PSOAM_FP16, true)
#undef PSOAM_SW16
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pack_r(const psoam_plan* P, const float* y, hipStream_t s) {
  const auto& g = P->g;
  if (P->d_f16) {
    hipError_t e = f16_amax(P, y, (int64_t)P->y_elems(), 1, s);
    if (e == hipSuccess) e = f16_scale(P, 1, 1.0, 0.0, s);
    if (e != hipSuccess) return e;
  }
  // 16-byte loads of the A-scans when every octet starts 16-byte aligned
  const int vec4 = ((uintptr_t)y & 15) == 0 && (g.nt & 3) == 0;
  switch (P->prec) {
    case PSOAM_FP32:
      hipLaunchKernelGGL(pack_r32, dim3(g.ny * g.nx), dim3(256), 0, s, y, (float*)P->d_rq,
                         g.n_pulses, g.ny, g.nx, g.nt, P->Lt, P->Kp, P->Xp, P->R, P->ps_r,
                         gate_now());
      break;
#define PSOAM_PK16(PR, SP)                                                                  \
  {                                                                                         \
    using E = Half<PR>::E;                                                                  \
    const size_t n = (size_t)g.ny * g.nx;                                                   \
    hipLaunchKernelGGL((pack_r16<PR, SP>), dim3((unsigned)n), dim3(256), 0, s, y,           \
                       (E*)P->d_rq, (E*)P->d_rq_lo, g.n_pulses, g.ny, g.nx, g.nt, P->Lt / 8, \
                       P->Kp, P->Xp, P->R, P->ps_r, vec4, P->tsh, P->d_f16, gate_now());    \
    break;                                                                                  \
  }
    case PSOAM_BF16:
    case PSOAM_BF16_REFINED: PSOAM_PK16(PSOAM_BF16, false)
    case PSOAM_FP16: PSOAM_PK16(PSOAM_FP16, false)
    case PSOAM_BF16_SPLIT: PSOAM_PK16(PSOAM_BF16, true)
    case PSOAM_FP16_SPLIT: PSOAM_PK16(PSOAM_FP16, true)
#undef PSOAM_PK16
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static bool use_lds(const psoam_plan* P, int mode) {
  const BandTable& T = (mode == 2) ? P->adj : P->fwd;
  return P->prec != PSOAM_FP32 && T.lds_ok;
}

static bool use_runs32(const psoam_plan* P, int mode) {
  const BandTable& T = (mode == 2) ? P->adj : P->fwd;
  return P->prec == PSOAM_FP32 && T.runs32;
}

static size_t band_blocks(const psoam_plan* P, int mode) {
  const BandTable& T = (mode == 2) ? P->adj : P->fwd;
  if (use_runs32(P, mode)) {
    const size_t nyb = (P->g.ny + kWavesPerBlock - 1) / kWavesPerBlock;
    const size_t nxb = (P->g.nx + kLdsPos - 1) / kLdsPos;
    return (size_t)T.n_mtiles * nyb * nxb;
  }
  if (use_lds(P, mode)) {
    // 8 ceil(npos / 8) blocks per tile (every XCD takes an equal share)
    const size_t nyb = (P->g.ny + T.rows - 1) / T.rows;
    const size_t nxb = (P->g.nx + kLdsPos - 1) / kLdsPos;
    return (size_t)T.n_mtiles * ((nyb * nxb + 7) / 8 * 8);
  }
  const int n_mblk = (T.n_mtiles + kWavesPerBlock - 1) / kWavesPerBlock;
  const int nxb = (P->g.nx + kPosPerWave - 1) / kPosPerWave;
  return (size_t)n_mblk * P->g.ny * nxb;
}

size_t band_partials(const psoam_plan* P, int mode) {
  const BandTable& T = (mode == 2) ? P->adj : P->fwd;
  return band_blocks(P, mode) * (use_lds(P, mode) ? T.rows : kWavesPerBlock);
}

template <int MODE>
static hipError_t launch_band_lds(const psoam_plan* P, const BandTable& T, BandArgs& A,
                                  dim3 grid, hipStream_t s) {
  LdsArgs L;
  L.lstart = T.d_lstart;
  L.order = T.d_order;
  L.rinfo = T.d_rinfo;
  L.max_runs = T.max_runs;
  L.lgrp = T.d_lgrp;
  L.win = T.d_win;
  L.la = T.d_la;
  L.la_lo = T.d_la_lo;
  L.la_bytes = (int)((size_t)(T.l_chunks + kRunMax) * kWaveLanes * 8 * sizeof(uint16_t));
  L.f = P->F;
  L.yp = P->Yp;
  L.nyb = (P->g.ny + T.rows - 1) / T.rows;
  L.nxb = (P->g.nx + kLdsPos - 1) / kLdsPos;
  L.lds_elems = (int)(T.lds_bytes / sizeof(uint16_t));
  L.meta_off = (int)((T.lds_bytes + 15) / 16 * 16);
  const size_t lds = L.meta_off + lds_meta_bytes(P->F, T.rows, T.max_runs);
#define PSOAM_LDS_K(PR, SP, R, PF)                                                          \
  {                                                                                         \
    if constexpr (MODE == 2) {                                                              \
      auto kern = band16_lds_adj<PR, SP, R, PF>;                                            \
      if (lds > 64 * 1024)                                                                  \
        (void)hipFuncSetAttribute((const void*)kern,                                        \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);    \
      hipLaunchKernelGGL(kern, grid, dim3(64 * (R + PF)), lds, s, A, L);                    \
    } else {                                                                                \
      auto kern = band16_lds<PR, SP, MODE, R, PF>;                                          \
      if (lds > 64 * 1024)                                                                  \
        (void)hipFuncSetAttribute((const void*)kern,                                        \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);    \
      hipLaunchKernelGGL(kern, grid, dim3(64 * (R + PF)), lds, s, A, L);                    \
    }                                                                                       \
  }
#define PSOAM_LDS_R(PR, SP, R) PSOAM_LDS_K(PR, SP, R, 0)
#define PSOAM_LDS(PR, SP)                                                                   \
  {                                                                                         \
    if (T.rows == 8) PSOAM_LDS_R(PR, SP, 8) else PSOAM_LDS_R(PR, SP, 4)                     \
    break;                                                                                  \
  }
  // 12-row workgroups: one-part operands only (the plan never picks them
  // for split ones)
#define PSOAM_LDS12(PR)                                                                     \
  {                                                                                         \
    if (T.rows == 12) PSOAM_LDS_R(PR, false, 12) else if (T.rows == 8) PSOAM_LDS_R(PR, false, 8) \
    else PSOAM_LDS_R(PR, false, 4)                                                          \
    break;                                                                                  \
  }
  // one-part operands, one 8-row workgroup per CU: four loader waves beside
  // the eight contracting ones (H and its residual form)
#define PSOAM_LDS_PF(PR)                                                                    \
  {                                                                                         \
    PSOAM_LDS_K(PR, false, 8, 4)                                                            \
    break;                                                                                  \
  }
  if constexpr (MODE != 2) {
  if (T.loadw > 0 && T.rows == 8) {
    switch (P->prec) {
      case PSOAM_BF16:
      case PSOAM_BF16_REFINED: PSOAM_LDS_PF(PSOAM_BF16)
      case PSOAM_FP16: PSOAM_LDS_PF(PSOAM_FP16)
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  }
#undef PSOAM_LDS_PF
  if (T.rows == 12 && (P->prec == PSOAM_BF16_SPLIT || P->prec == PSOAM_FP16_SPLIT))
    return hipErrorInvalidValue;
  switch (P->prec) {
    case PSOAM_BF16:
    case PSOAM_BF16_REFINED: PSOAM_LDS12(PSOAM_BF16)
    case PSOAM_FP16: PSOAM_LDS12(PSOAM_FP16)
    case PSOAM_BF16_SPLIT: PSOAM_LDS(PSOAM_BF16, true)
    case PSOAM_FP16_SPLIT: PSOAM_LDS(PSOAM_FP16, true)
    default:
      return hipErrorInvalidValue;
  }
#undef PSOAM_LDS12
#undef PSOAM_LDS
#undef PSOAM_LDS_R
#undef PSOAM_LDS_K
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_band_mode(const psoam_plan* P, BandArgs& A, dim3 grid, hipStream_t s) {
  const int NB = P->NB;
#define PSOAM_NB_CASES(KERNEL_T)                                                        \
  switch (NB) {                                                                         \
    case 1: hipLaunchKernelGGL((KERNEL_T<1, MODE>), grid, dim3(256), 0, s, A); break;   \
    case 2: hipLaunchKernelGGL((KERNEL_T<2, MODE>), grid, dim3(256), 0, s, A); break;   \
    case 3: hipLaunchKernelGGL((KERNEL_T<3, MODE>), grid, dim3(256), 0, s, A); break;   \
    case 4: hipLaunchKernelGGL((KERNEL_T<4, MODE>), grid, dim3(256), 0, s, A); break;   \
    default: return hipErrorInvalidValue;                                               \
  }
  switch (P->prec) {
    case PSOAM_FP32: {
      PSOAM_NB_CASES(band32)
      break;
    }
#define PSOAM_B16(PR, SP)                                                                   \
  {                                                                                         \
    switch (NB) {                                                                           \
      case 1: hipLaunchKernelGGL((band16<PR, SP, 1, MODE>), grid, dim3(256), 0, s, A); break; \
      case 2: hipLaunchKernelGGL((band16<PR, SP, 2, MODE>), grid, dim3(256), 0, s, A); break; \
      case 3: hipLaunchKernelGGL((band16<PR, SP, 3, MODE>), grid, dim3(256), 0, s, A); break; \
      case 4: hipLaunchKernelGGL((band16<PR, SP, 4, MODE>), grid, dim3(256), 0, s, A); break; \
      default: return hipErrorInvalidValue;                                                 \
    }                                                                                       \
    break;                                                                                  \
  }
    case PSOAM_BF16:
    case PSOAM_BF16_REFINED: PSOAM_B16(PSOAM_BF16, false)
    case PSOAM_FP16: PSOAM_B16(PSOAM_FP16, false)
    case PSOAM_BF16_SPLIT: PSOAM_B16(PSOAM_BF16, true)
    case PSOAM_FP16_SPLIT: PSOAM_B16(PSOAM_FP16, true)
#undef PSOAM_B16
    default:
      return hipErrorInvalidValue;
  }
#undef PSOAM_NB_CASES
  return hipGetLastError();
}

hipError_t launch_band(const psoam_plan* P, int mode, float* out, const float* pmeas,
                       double* partial, hipStream_t s, float* yc, double yc_beta, int yc_first) {
  // the residual form with the A c recurrence is a kernel form of its own
  // (mode 3), so the plain residual form carries none of its registers
  if (mode == 1 && yc) mode = 3;
  const BandTable& T = (mode == 2) ? P->adj : P->fwd;
  const bool split = P->prec == PSOAM_BF16_SPLIT || P->prec == PSOAM_FP16_SPLIT;
  const bool fp16 = P->prec == PSOAM_FP16 || P->prec == PSOAM_FP16_SPLIT;
  BandArgs A;
  A.q = (mode == 2) ? P->d_rq : P->d_bq;
  A.q_lo = (mode == 2) ? P->d_rq_lo : P->d_bq_lo;
  A.start = T.d_start;
  A.off = T.d_off;
  A.a = T.d_a;
  A.a_lo = split ? T.d_a_lo : nullptr;
  A.n_mtiles = T.n_mtiles;
  A.n_mblk = (T.n_mtiles + kWavesPerBlock - 1) / kWavesPerBlock;
  A.ny = P->g.ny;
  A.nx = P->g.nx;
  A.nxb = (P->g.nx + kPosPerWave - 1) / kPosPerWave;
  A.m_rows = T.m_rows;
  A.xp = P->Xp;
  A.ps = (mode == 2) ? P->ps_r : P->ps_b;
  A.nk = P->g.n_pulses;
  A.kp = P->Kp;
  A.half = T.half;
  A.inv_scale = fp16 ? 1.0f / kFp16Scale : 1.0f;
  A.f16 = P->d_f16;
  A.gate = gate_now();
  if ((mode == 1 || mode == 3) && P->d_f16) {
    // residual r = H b - p: |r| <= hrow max |b| + max |p| with max |b| <= srow max |x|
    const hipError_t e = f16_scale(P, 3, P->hrow * P->srow, 1.0, s);
    if (e != hipSuccess) return e;
  }
  A.out = out;
  A.pmeas = pmeas;
  A.rq = P->d_rq;
  A.rq_lo = P->d_rq_lo;
  A.ps_r = P->ps_r;
  A.r = P->R;
  A.tsh = P->tsh;
  A.rq_scale = fp16 ? kFp16Scale : 1.0f;
  A.partial = partial;
  A.yc = mode == 3 ? yc : nullptr;
  A.yc_beta = (float)yc_beta;
  A.yc_inv = (float)(1.0 / (1.0 + yc_beta));
  A.yc_first = yc_first;
  A.sw = P->sw;
  A.phi = P->d_phi;
  A.stab = P->d_stab;
  A.nz = P->g.nz;
  A.nt = P->g.nt;
  const dim3 grid((unsigned)band_blocks(P, mode));
  (void)split;
  if (use_runs32(P, mode)) {
    LdsArgs L{};
    L.lstart = T.d_lstart;
    L.lgrp = T.d_lgrp;
    L.la = T.d_la;
    L.order = T.d_order;
    L.rinfo = T.d_rinfo;
    L.f = P->F;
    L.nyb = (P->g.ny + kWavesPerBlock - 1) / kWavesPerBlock;
    L.nxb = (P->g.nx + kLdsPos - 1) / kLdsPos;
    L.la_bytes = (int)((size_t)(T.l_chunks + kRunMax) * kWaveLanes * sizeof(float));
    const dim3 blk(64 * kWavesPerBlock);
    switch (mode) {
      case 0: hipLaunchKernelGGL(band32_run<0>, grid, blk, 0, s, A, L); break;
      case 1: hipLaunchKernelGGL(band32_run<1>, grid, blk, 0, s, A, L); break;
      case 2: hipLaunchKernelGGL(band32_run<2>, grid, blk, 0, s, A, L); break;
      case 3: hipLaunchKernelGGL(band32_run<3>, grid, blk, 0, s, A, L); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (use_lds(P, mode)) {
    switch (mode) {
      case 0: return launch_band_lds<0>(P, T, A, grid, s);
      case 1: return launch_band_lds<1>(P, T, A, grid, s);
      case 2: return launch_band_lds<2>(P, T, A, grid, s);
      case 3: return launch_band_lds<3>(P, T, A, grid, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (mode) {
    case 0: return launch_band_mode<0>(P, A, grid, s);
    case 1: return launch_band_mode<1>(P, A, grid, s);
    case 2: return launch_band_mode<2>(P, A, grid, s);
    case 3: return launch_band_mode<3>(P, A, grid, s);
    default: return hipErrorInvalidValue;
  }
}

// --------------------------------------------------------------------------
// elementwise and prox kernels
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void prox_l1_kernel(float* __restrict__ x,
                                                      const float* __restrict__ z, int64_t n,
                                                      float th, int nonneg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = z[i];
  if (nonneg) {
    x[i] = fmaxf(v - th, 0.0f);
  } else {
    const float m = fmaxf(fabsf(v) - th, 0.0f);
    x[i] = copysignf(m, v) * (m > 0.0f ? 1.0f : 0.0f);
  }
}

hipError_t launch_prox_l1(float* x, const float* z, int64_t n, float thresh, int nonneg,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(prox_l1_kernel, dim3(blocks_for((size_t)n)), dim3(256), 0, s, x, z, n,
                     thresh, nonneg);
  return hipGetLastError();
}

struct Grid3 {
  int ny, nx, nz;
  int64_t sv;  // S * V
  const int* gate;  // device stop flag of the solve, or null
};

__device__ __forceinline__ float eta_at(const float* __restrict__ uc, const float* __restrict__ up,
                                        float beta, int64_t i) {
  if (!uc) return 0.0f;
  const float a = uc[i];
  return up ? a + beta * (a - up[i]) : a;
}

// (grad^T eta)[v] for component arrays laid out [3][S*V]
__device__ __forceinline__ float gradT_at(const float* __restrict__ uc, const float* __restrict__ up,
                                          float beta, const Grid3& G, int64_t v, int y, int x,
                                          int z) {
  const int64_t sx = G.nz, sy = (int64_t)G.nx * G.nz;
  float acc = 0.0f;
  // component 0: differences along y
  if (y > 0) acc += eta_at(uc, up, beta, v - sy);
  if (y < G.ny - 1) acc -= eta_at(uc, up, beta, v);
  // component 1: along x
  const float* uc1 = uc ? uc + G.sv : nullptr;
  const float* up1 = up ? up + G.sv : nullptr;
  if (x > 0) acc += eta_at(uc1, up1, beta, v - sx);
  if (x < G.nx - 1) acc -= eta_at(uc1, up1, beta, v);
  // component 2: along z
  const float* uc2 = uc ? uc + 2 * G.sv : nullptr;
  const float* up2 = up ? up + 2 * G.sv : nullptr;
  if (z > 0) acc += eta_at(uc2, up2, beta, v - 1);
  if (z < G.nz - 1) acc -= eta_at(uc2, up2, beta, v);
  return acc;
}

// One dual step of the TV prox, fused:
//   eta = u_j + beta (u_j - u_{j-1}),  w = z - grad^T eta,
//   u_{j+1} = clamp(eta + inv_mu grad w, -theta, theta)   (per component).
// A block owns a TY x TX x TZ tile of one species volume.  eta is staged in
// LDS per component over the tile, its forward halo and the one backward
// plane that component's difference needs; w is formed on the tile plus the
// forward halo; the new duals are written for the tile.  Global traffic is
// about u_j, u_{j-1} (3 components each), z in and u_{j+1} out per voxel.
// Every output is the same expression of the same inputs whatever the tile,
// so the tile shape (chosen per plan by the autotuner) never changes results.
template <int Y, int X, int Z>
struct Dims3 {
  static constexpr int y = Y, x = X, z = Z;
};
// tile shapes (y, x, z, threads); entry 0 is the default
constexpr int kTvTiles = 5;
constexpr int kTvTile[kTvTiles][4] = {
    {8, 8, 32, 512}, {4, 8, 32, 256}, {4, 16, 32, 512}, {4, 8, 64, 512}, {8, 8, 32, 1024}};
int tv_tile_count() { return kTvTiles; }
void tv_tile_dims(int i, int* d) {
  for (int k = 0; k < 4; ++k) d[k] = kTvTile[i][k];
}

template <int kTvY, int kTvX, int kTvZ, int kTvThreads>
__global__ __launch_bounds__(kTvThreads) void tv_step_kernel(float* __restrict__ un,
                                                      const float* __restrict__ zin,
                                                      const float* __restrict__ uc,
                                                      const float* __restrict__ up, float beta,
                                                      float inv_mu, float theta, Grid3 G) {
  if (G.gate && *G.gate) return;  // a device stop test has ended the solve
  constexpr int EY = kTvY + 1, EX = kTvX + 1, EZ = kTvZ + 1;  // w region (tile + forward halo)
  __shared__ float s_ey[(EY + 1) * EX * EZ];  // eta_y, y from y0 - 1
  __shared__ float s_ex[EY * (EX + 1) * EZ];  // eta_x, x from x0 - 1
  __shared__ float s_ez[EY * EX * (EZ + 1)];  // eta_z, z from z0 - 1
  __shared__ float s_w[EY * EX * EZ];
  const int nzb = (G.nz + kTvZ - 1) / kTvZ, nxb = (G.nx + kTvX - 1) / kTvX;
  const int nyb = (G.ny + kTvY - 1) / kTvY;
  // a tile's z, x and y neighbours (whose duals it reads as halo) mostly run
  // from the same L2
  int bb = xcd_block();
  const int zb = bb % nzb;
  bb /= nzb;
  const int xb = bb % nxb;
  bb /= nxb;
  const int yb = bb % nyb;
  const int sp = bb / nyb;
  const int y0 = yb * kTvY, x0 = xb * kTvX, z0 = zb * kTvZ;
  const int64_t vol = (int64_t)G.ny * G.nx * G.nz;
  const int64_t sbase = (int64_t)sp * vol;
  const int tid = threadIdx.x;
  // eta of component d on a region of NY_ x NX_ x NZ_ points from (gy0, gx0, gz0)
  // into LDS: all of a thread's loads are issued before any is used
  auto stage = [&](float* dst, int d, auto dims, int gy0, int gx0, int gz0) {
    constexpr int NY_ = decltype(dims)::y, NX_ = decltype(dims)::x, NZ_ = decltype(dims)::z;
    constexpr int CNT = NY_ * NX_ * NZ_;
    constexpr int IT = (CNT + kTvThreads - 1) / kTvThreads;
    const float* c = uc ? uc + d * G.sv : nullptr;
    const float* pr = up ? up + d * G.sv : nullptr;
    float a[IT], b[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = tid + it * kTvThreads;
      const int lz = i % NZ_, r = i / NZ_;
      const int lx = r % NX_, ly = r / NX_;
      const int gy = gy0 + ly, gx = gx0 + lx, gz = gz0 + lz;
      a[it] = 0.0f;
      b[it] = 0.0f;
      if (c && i < CNT && gy >= 0 && gy < G.ny && gx >= 0 && gx < G.nx && gz >= 0 && gz < G.nz) {
        const int64_t v = sbase + ((int64_t)gy * G.nx + gx) * G.nz + gz;
        a[it] = c[v];
        if (pr) b[it] = pr[v];
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = tid + it * kTvThreads;
      if (i < CNT) dst[i] = pr ? a[it] + beta * (a[it] - b[it]) : a[it];
    }
  };
  stage(s_ey, 0, Dims3<EY + 1, EX, EZ>{}, y0 - 1, x0, z0);
  stage(s_ex, 1, Dims3<EY, EX + 1, EZ>{}, y0, x0 - 1, z0);
  stage(s_ez, 2, Dims3<EY, EX, EZ + 1>{}, y0, x0, z0 - 1);
  __syncthreads();
  // w on the tile and its forward halo (the z loads first, then the sums)
  constexpr int WIT = (EY * EX * EZ + kTvThreads - 1) / kTvThreads;
  float zv[WIT];
#pragma unroll
  for (int it = 0; it < WIT; ++it) {
    const int i = tid + it * kTvThreads;
    const int lz = i % EZ, r = i / EZ;
    const int lx = r % EX, ly = r / EX;
    const int gy = y0 + ly, gx = x0 + lx, gz = z0 + lz;
    zv[it] = (i < EY * EX * EZ && gy < G.ny && gx < G.nx && gz < G.nz)
                 ? zin[sbase + ((int64_t)gy * G.nx + gx) * G.nz + gz]
                 : 0.0f;
  }
#pragma unroll
  for (int it = 0; it < WIT; ++it) {
    const int i = tid + it * kTvThreads;
    if (i >= EY * EX * EZ) break;
    const int lz = i % EZ, r = i / EZ;
    const int lx = r % EX, ly = r / EX;
    const int gy = y0 + ly, gx = x0 + lx, gz = z0 + lz;
    float wv = 0.0f;
    if (gy < G.ny && gx < G.nx && gz < G.nz) {
      float acc = 0.0f;
      if (gy > 0) acc += s_ey[(ly * EX + lx) * EZ + lz];
      if (gy < G.ny - 1) acc -= s_ey[((ly + 1) * EX + lx) * EZ + lz];
      if (gx > 0) acc += s_ex[(ly * (EX + 1) + lx) * EZ + lz];
      if (gx < G.nx - 1) acc -= s_ex[(ly * (EX + 1) + lx + 1) * EZ + lz];
      if (gz > 0) acc += s_ez[(ly * EX + lx) * (EZ + 1) + lz];
      if (gz < G.nz - 1) acc -= s_ez[(ly * EX + lx) * (EZ + 1) + lz + 1];
      wv = zv[it] - acc;
    }
    s_w[i] = wv;
  }
  __syncthreads();
  // new duals on the tile
  for (int i = tid; i < kTvY * kTvX * kTvZ; i += kTvThreads) {
    const int lz = i % kTvZ, r = i / kTvZ;
    const int lx = r % kTvX, ly = r / kTvX;
    const int gy = y0 + ly, gx = x0 + lx, gz = z0 + lz;
    if (gy >= G.ny || gx >= G.nx || gz >= G.nz) continue;
    const int wi = (ly * EX + lx) * EZ + lz;
    const float wv = s_w[wi];
    const float gyd = gy < G.ny - 1 ? s_w[wi + EX * EZ] - wv : 0.0f;
    const float gxd = gx < G.nx - 1 ? s_w[wi + EZ] - wv : 0.0f;
    const float gzd = gz < G.nz - 1 ? s_w[wi + 1] - wv : 0.0f;
    const float ey = s_ey[((ly + 1) * EX + lx) * EZ + lz];
    const float ex = s_ex[(ly * (EX + 1) + lx + 1) * EZ + lz];
    const float ez = s_ez[(ly * EX + lx) * (EZ + 1) + lz + 1];
    const int64_t v = sbase + ((int64_t)gy * G.nx + gx) * G.nz + gz;
    un[v] = fminf(fmaxf(ey + inv_mu * gyd, -theta), theta);
    un[G.sv + v] = fminf(fmaxf(ex + inv_mu * gxd, -theta), theta);
    un[2 * G.sv + v] = fminf(fmaxf(ez + inv_mu * gzd, -theta), theta);
  }
}

__global__ __launch_bounds__(256) void tv_final_kernel(float* __restrict__ x,
                                                       const float* __restrict__ z,
                                                       const float* __restrict__ u, int mode,
                                                       float th1, Grid3 G) {
  if (G.gate && *G.gate) return;  // a device stop test has ended the solve
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= G.sv) return;
  const int iz = (int)(v % G.nz);
  const int ix = (int)((v / G.nz) % G.nx);
  const int iy = (int)((v / ((int64_t)G.nz * G.nx)) % G.ny);
  float r = z[v] - gradT_at(u, nullptr, 0.0f, G, v, iy, ix, iz);
  if (mode == 1) r = fmaxf(r, 0.0f);
  if (mode == 2) r = fmaxf(r - th1, 0.0f);
  x[v] = r;
}

static Grid3 grid3(const psoam_plan* P) {
  Grid3 G;
  G.ny = P->g.ny;
  G.nx = P->g.nx;
  G.nz = P->g.nz;
  G.sv = (int64_t)P->c_elems();
  G.gate = gate_now();
  return G;
}

hipError_t launch_tv_step(const psoam_plan* P, float* u_next, const float* z, const float* u_cur,
                          const float* u_prev, float beta, float inv_mu, float theta,
                          hipStream_t s) {
  const Grid3 G = grid3(P);
  const int t = P->tv_tile >= 0 && P->tv_tile < kTvTiles ? P->tv_tile : 0;
  const int* d = kTvTile[t];
  const size_t nb = (size_t)P->g.n_species * ((G.ny + d[0] - 1) / d[0]) *
                    ((G.nx + d[1] - 1) / d[1]) * ((G.nz + d[2] - 1) / d[2]);
  if (nb == 0) return hipSuccess;
#define PSOAM_TV(I)                                                                          \
  case I:                                                                                    \
    hipLaunchKernelGGL((tv_step_kernel<kTvTile[I][0], kTvTile[I][1], kTvTile[I][2],          \
                                       kTvTile[I][3]>),                                      \
                       dim3((unsigned)nb), dim3(kTvTile[I][3]), 0, s, u_next, z, u_cur, u_prev, \
                       beta, inv_mu, theta, G);                                              \
    break;
  switch (t) {
    PSOAM_TV(0)
    PSOAM_TV(1)
    PSOAM_TV(2)
    PSOAM_TV(3)
    PSOAM_TV(4)
    default:
      return hipErrorInvalidValue;
  }
#undef PSOAM_TV
  return hipGetLastError();
}

hipError_t launch_tv_final(const psoam_plan* P, float* x, const float* z, const float* u,
                           int mode, float thresh1, hipStream_t s) {
  const Grid3 G = grid3(P);
  hipLaunchKernelGGL(tv_final_kernel, dim3(blocks_for((size_t)G.sv)), dim3(256), 0, s, x, z, u,
                     mode, thresh1, G);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void axpby_kernel(float* __restrict__ out,
                                                    const float* __restrict__ x,
                                                    const float* __restrict__ y, float a,
                                                    float b, int64_t n,
                                                    const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * x[i] + b * y[i];
}

hipError_t launch_axpby(float* out, const float* x, const float* y, float a, float b, int64_t n,
                        hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(axpby_kernel, dim3(blocks_for((size_t)n)), dim3(256), 0, s, out, x, y, a, b,
                     n, gate_now());
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_kernel(float* __restrict__ x, float v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

hipError_t launch_fill(float* x, float v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for((size_t)n)), dim3(256), 0, s, x, v, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- reductions
constexpr int kRedBlocks = 1024;

size_t reduce_blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (size_t)(b < kRedBlocks ? (b > 0 ? b : 1) : kRedBlocks);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void dot_kernel(const float* __restrict__ x,
                                                  const float* __restrict__ y, int64_t n,
                                                  double* __restrict__ partial,
                                                  const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  __shared__ double sh[4];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    acc += (double)x[i] * (double)y[i];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ partial,
                                                           int64_t n, double* __restrict__ out,
                                                           const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  __shared__ double sh[4];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += partial[i];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = r;
}

hipError_t launch_dot(const float* x, const float* y, int64_t n, double* partial, double* out,
                      hipStream_t s) {
  const size_t nb = reduce_blocks(n);
  hipLaunchKernelGGL(dot_kernel, dim3((unsigned)nb), dim3(256), 0, s, x, y, n, partial, gate_now());
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partial, (int64_t)nb, out,
                     gate_now());
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partial, size_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partial, (int64_t)n, out,
                     gate_now());
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void tv_l1_kernel(const float* __restrict__ c, Grid3 G,
                                                    double* __restrict__ partial) {
  if (G.gate && *G.gate) return;  // a device stop test has ended the solve
  __shared__ double sh[4];
  double tvs = 0.0, l1 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t sx = G.nz, sy = (int64_t)G.nx * G.nz;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < G.sv; v += stride) {
    const int iz = (int)(v % G.nz);
    const int ix = (int)((v / G.nz) % G.nx);
    const int iy = (int)((v / ((int64_t)G.nz * G.nx)) % G.ny);
    const float cv = c[v];
    l1 += fabs((double)cv);
    if (iy < G.ny - 1) tvs += fabs((double)c[v + sy] - (double)cv);
    if (ix < G.nx - 1) tvs += fabs((double)c[v + sx] - (double)cv);
    if (iz < G.nz - 1) tvs += fabs((double)c[v + 1] - (double)cv);
  }
  const double r0 = block_sum(tvs, sh);
  const double r1 = block_sum(l1, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = r0;
    partial[gridDim.x + blockIdx.x] = r1;
  }
}

hipError_t launch_tv_l1_sums(const psoam_plan* P, const float* c, double* partial, double* out,
                             hipStream_t s) {
  const Grid3 G = grid3(P);
  const size_t nb = reduce_blocks(G.sv);
  hipLaunchKernelGGL(tv_l1_kernel, dim3((unsigned)nb), dim3(256), 0, s, c, G, partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partial, (int64_t)nb, out,
                     gate_now());
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partial + nb, (int64_t)nb,
                     out + 1, gate_now());
  return hipGetLastError();
}

// ---- full regulariser with the TV(S c) term: stacked dual iteration -------
// Duals: u1 [3][S][V] (differences of c), u2 [3][K][V] (differences of each
// pulse image S c), u3 [S][V] (the l1 block); eta = u_c + beta (u_c - u_p),
// with u_c == null meaning eta = 0 and u_p == null meaning eta = u_c.
__device__ __forceinline__ float eta3(const float* __restrict__ uc, const float* __restrict__ up,
                                      float beta, int64_t i) {
  if (!uc) return 0.0f;
  const float a = uc[i];
  return up ? a + beta * (a - up[i]) : a;
}

// eta of four pulses at once (u2 is stored in groups of four pulses, see below)
__device__ __forceinline__ f32x4 eta4(const f32x4* __restrict__ uc, const f32x4* __restrict__ up,
                                      float beta, int64_t i) {
  if (!uc) return f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const f32x4 a = uc[i];
  if (!up) return a;
  const f32x4 b = up[i];
  f32x4 r;
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = a[q] + beta * (a[q] - b[q]);
  return r;
}

// u2 layout: [3][ceil(K/4)][V][4], pulse k of direction d at voxel v in float
// ((d * ceil(K/4) + k / 4) * V + v) * 4 + k % 4, so a thread reads the duals
// of four pulses with one 16-byte load (consecutive voxels stay consecutive
// 16-byte words); the padding pulses of the last group are kept at zero.
//
// S^T grad^T eta2 needs eta2 at v and at its backward neighbours, summed over
// the pulses with the coefficients of v.  Both S^T and grad^T are linear, so
// the update kernel that produces eta2 also reduces it over the pulses
// (projections, [6][S][V]):
//   slot d     (d = y, x, z): A_d[s][v] = sum_k S_v[k][s] eta2_d[k][v]
//   slot 3 + d:               B_d[s][v] = sum_k S_{v + e_d}[k][s] eta2_d[k][v]
// so that (S^T grad^T eta2)[s][v] = sum_d ([i_d > 0] B_d[s][v - e_d]
// - [i_d < n_d - 1] A_d[s][v]).  With a per-depth table the y and x
// neighbours share v's coefficients (B_y = A_y, B_x = A_x; slots 3 and 4 are
// not written).  u2 is then read once per dual step (current and previous)
// and written once, instead of being read again for w.
__device__ __forceinline__ int r3_bslot(bool depth_table, int d) {
  return (depth_table && d < 2) ? d : 3 + d;
}

// w = z - (grad^T eta1 + S^T grad^T eta2 + eta3); with clamp_out the
// algorithm's output max(., 0) instead.  eta2 enters through its projections
// pq (null: eta2 = 0).  One thread per voxel position, all species.
__global__ __launch_bounds__(256) void r3_w_kernel(
    float* __restrict__ out, const float* __restrict__ z, const float* __restrict__ u1c,
    const float* __restrict__ u1p, const float* __restrict__ pq, const float* __restrict__ u3c,
    const float* __restrict__ u3p, float beta, int ns, int depth_table, Grid3 G, int clamp_out) {
  if (G.gate && *G.gate) return;  // a device stop test has ended the solve
  const int64_t vol = (int64_t)G.ny * G.nx * G.nz;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= vol) return;
  const int iz = (int)(v % G.nz);
  const int ix = (int)((v / G.nz) % G.nx);
  const int iy = (int)(v / ((int64_t)G.nz * G.nx));
  const int idx[3] = {iy, ix, iz};
  const int nd[3] = {G.ny, G.nx, G.nz};
  const int64_t st[3] = {(int64_t)G.nx * G.nz, G.nz, 1};
  for (int s = 0; s < ns; ++s) {
    float gt = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t base = ((int64_t)d * ns + s) * vol;
      if (idx[d] > 0) gt += eta3(u1c, u1p, beta, base + v - st[d]);
      if (idx[d] < nd[d] - 1) gt -= eta3(u1c, u1p, beta, base + v);
      if (pq) {
        const int64_t bb = ((int64_t)r3_bslot(depth_table, d) * ns + s) * vol;
        if (idx[d] > 0) gt += pq[bb + v - st[d]];
        if (idx[d] < nd[d] - 1) gt -= pq[base + v];
      }
    }
    const int64_t i = (int64_t)s * vol + v;
    const float r = z[i] - (gt + eta3(u3c, u3p, beta, i));
    out[i] = clamp_out ? fmaxf(r, 0.0f) : r;
  }
}

// u1' = clip(eta1 + s1 grad w), u2' = clip(eta2 + s2 grad (S w)),
// u3' = clip(eta3 + s3 w), each at its own radius; one thread per voxel
// position (forward differences, zero at the last index of each axis).  Also
// writes the projections pq of the next step's eta2 = u2' + beta_next (u2' -
// u2) (beta_next = 0 on the last step: the projections of u2' itself).  NSM
// bounds the species count for the register arrays.
template <int NSM>
__global__ __launch_bounds__(256) void r3_u_kernel(
    float* __restrict__ n1, float* __restrict__ n2, float* __restrict__ n3,
    float* __restrict__ pq, const float* __restrict__ w, const float* __restrict__ u1c,
    const float* __restrict__ u1p, const float* __restrict__ u2c, const float* __restrict__ u2p,
    const float* __restrict__ u3c, const float* __restrict__ u3p, float beta, float beta_next,
    float s1, float s2, float s3, float th1, float th2, float th3, SwitchParams sw,
    const float* __restrict__ phi, const float* __restrict__ stab, Grid3 G) {
  if (G.gate && *G.gate) return;  // a device stop test has ended the solve
  const int64_t vol = (int64_t)G.ny * G.nx * G.nz;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= vol) return;
  const int iz = (int)(v % G.nz);
  const int ix = (int)((v / G.nz) % G.nx);
  const int iy = (int)(v / ((int64_t)G.nz * G.nx));
  const bool fwd[3] = {iy < G.ny - 1, ix < G.nx - 1, iz < G.nz - 1};
  const int64_t st[3] = {(int64_t)G.nx * G.nz, G.nz, 1};
  const int ns = sw.ns, nk = sw.nk;
  // w at v and at its three forward neighbours
  float wv[4][NSM];
#pragma unroll
  for (int s = 0; s < NSM; ++s) {
    wv[0][s] = wv[1][s] = wv[2][s] = wv[3][s] = 0.0f;
    if (s >= ns) continue;
    const int64_t i = (int64_t)s * vol + v;
    wv[0][s] = w[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) wv[d + 1][s] = fwd[d] ? w[i + st[d]] : 0.0f;
  }
#pragma unroll
  for (int s = 0; s < NSM; ++s) {
    if (s >= ns) continue;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t i = ((int64_t)d * ns + s) * vol + v;
      const float g = fwd[d] ? wv[d + 1][s] - wv[0][s] : 0.0f;
      n1[i] = fminf(fmaxf(eta3(u1c, u1p, beta, i) + s1 * g, -th1), th1);
    }
    const int64_t i = (int64_t)s * vol + v;
    n3[i] = fminf(fmaxf(eta3(u3c, u3p, beta, i) + s3 * wv[0][s], -th3), th3);
  }
  // coefficients at v and at its forward neighbours, generated in registers:
  // S_v[k][s] = phi_v (a_s + b_s e_s^k) with e_s = exp(-phi_v^gamma / tau_s);
  // e_s^k is taken from exp at the first pulse of each group of four and
  // multiplied by e_s within the group.  With a per-depth fluence the y and x
  // neighbours share v's coefficients.
  const bool depth_table = stab != nullptr;
  const size_t col0 = (size_t)v - iz;
  float ph[4];
  if (depth_table) {
    ph[0] = ph[1] = ph[2] = phi[iz];
    ph[3] = phi[fwd[2] ? iz + 1 : iz];
  } else {
    ph[0] = phi[col0 + iz];
    ph[1] = fwd[0] ? phi[col0 + st[0] + iz] : ph[0];
    ph[2] = fwd[1] ? phi[col0 + st[1] + iz] : ph[0];
    ph[3] = fwd[2] ? phi[col0 + iz + 1] : ph[0];
  }
  float rate[4][NSM];  // phi^gamma / tau_s per position
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float pg = (sw.gamma == 0.0f) ? 1.0f : powf(ph[j], sw.gamma);
#pragma unroll
    for (int s = 0; s < NSM; ++s) rate[j][s] = s < ns ? pg * sw.inv_tau[s] : 0.0f;
  }
  float pa[3][NSM], pb[3][NSM];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int s = 0; s < NSM; ++s) pa[d][s] = pb[d][s] = 0.0f;
  // u2 in groups of four pulses (layout above r3_w_kernel)
  const int nk4 = (nk + 3) >> 2;
  const f32x4* c4 = (const f32x4*)u2c;
  const f32x4* p4 = (const f32x4*)u2p;
  f32x4* o4 = (f32x4*)n2;
  for (int kg = 0; kg < nk4; ++kg) {
    f32x4 a[3], e[3], r[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t i = ((int64_t)d * nk4 + kg) * vol + v;
      a[d] = c4 ? c4[i] : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      e[d] = eta4(c4, p4, beta, i);
    }
    float ek[4][NSM], ef[4][NSM];  // e_s^k at the group's first pulse, e_s
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int s = 0; s < NSM; ++s) {
        ek[j][s] = expf(-(float)(kg * 4) * rate[j][s]);
        ef[j][s] = expf(-rate[j][s]);
      }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = kg * 4 + q;
      if (k >= nk) {
#pragma unroll
        for (int d = 0; d < 3; ++d) r[d][q] = 0.0f;
        continue;
      }
      float cs[NSM], cf[3][NSM];
      float sq0 = 0.0f, sqd[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s = 0; s < NSM; ++s) {
        cs[s] = cf[0][s] = cf[1][s] = cf[2][s] = 0.0f;
        if (s >= ns) continue;
        if (sw.diag) {
          cs[s] = k == s ? ph[0] : 0.0f;
#pragma unroll
          for (int d = 0; d < 3; ++d) cf[d][s] = (fwd[d] && k == s) ? ph[d + 1] : 0.0f;
        } else {
          cs[s] = ph[0] * (sw.a[s] + sw.b[s] * ek[0][s]);
#pragma unroll
          for (int d = 0; d < 3; ++d)
            cf[d][s] = fwd[d] ? ph[d + 1] * (sw.a[s] + sw.b[s] * ek[d + 1][s]) : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) ek[j][s] *= ef[j][s];
        sq0 += cs[s] * wv[0][s];
#pragma unroll
        for (int d = 0; d < 3; ++d) sqd[d] += cf[d][s] * wv[d + 1][s];
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float g = fwd[d] ? sqd[d] - sq0 : 0.0f;
        const float un = fminf(fmaxf(e[d][q] + s2 * g, -th2), th2);
        r[d][q] = un;
        const float en = un + beta_next * (un - a[d][q]);
#pragma unroll
        for (int s = 0; s < NSM; ++s) {
          pa[d][s] += cs[s] * en;
          pb[d][s] += cf[d][s] * en;
        }
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) o4[((int64_t)d * nk4 + kg) * vol + v] = r[d];
  }
#pragma unroll
  for (int s = 0; s < NSM; ++s) {
    if (s >= ns) continue;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      pq[((int64_t)d * ns + s) * vol + v] = pa[d][s];
      if (!depth_table || d == 2) pq[((int64_t)(3 + d) * ns + s) * vol + v] = pb[d][s];
    }
  }
}

// sum over pulses and positions of |differences of S c| (TV of S c), FP64
// partial sums per block
__global__ __launch_bounds__(256) void tvs_kernel(const float* __restrict__ c, SwitchParams sw,
                                                  const float* __restrict__ phi,
                                                  const float* __restrict__ stab, int kp, Grid3 G,
                                                  double* __restrict__ partial) {
  if (G.gate && *G.gate) return;  // a device stop test has ended the solve
  __shared__ double sh[4];
  const int64_t vol = (int64_t)G.ny * G.nx * G.nz;
  const int64_t st[3] = {(int64_t)G.nx * G.nz, G.nz, 1};
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < vol; v += stride) {
    const int iz = (int)(v % G.nz);
    const int ix = (int)((v / G.nz) % G.nx);
    const int iy = (int)(v / ((int64_t)G.nz * G.nx));
    const bool fwd[3] = {iy < G.ny - 1, ix < G.nx - 1, iz < G.nz - 1};
    const size_t col0 = (size_t)v - iz;
    const size_t colq[3] = {col0 + (size_t)st[0], col0 + (size_t)st[1], col0};
    const int zq[3] = {iz, iz, iz + 1};
    for (int k = 0; k < sw.nk; ++k) {
      double b0 = 0.0;
      for (int s = 0; s < sw.ns; ++s)
        b0 += (double)coef_zt(sw, phi, stab, G.nz, col0, iz, k, s) * (double)c[(int64_t)s * vol + v];
      for (int d = 0; d < 3; ++d) {
        if (!fwd[d]) continue;
        double bd = 0.0;
        for (int s = 0; s < sw.ns; ++s)
          bd += (double)coef_zt(sw, phi, stab, G.nz, colq[d], zq[d], k, s) *
                (double)c[(int64_t)s * vol + v + st[d]];
        acc += fabs(bd - b0);
      }
    }
  }
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

hipError_t launch_r3_w(const psoam_plan* P, float* out, const float* z, const float* u1c,
                       const float* u1p, const float* pq, const float* u3c, const float* u3p,
                       float beta, int clamp_out, hipStream_t s) {
  const Grid3 G = grid3(P);
  const size_t vol = P->v_elems();
  if (vol == 0) return hipSuccess;
  hipLaunchKernelGGL(r3_w_kernel, dim3(blocks_for(vol)), dim3(256), 0, s, out, z, u1c, u1p, pq,
                     u3c, u3p, beta, P->sw.ns, P->d_stab_t ? 1 : 0, G, clamp_out);
  return hipGetLastError();
}

hipError_t launch_r3_u(const psoam_plan* P, float* n1, float* n2, float* n3, float* pq,
                       const float* w, const float* u1c, const float* u1p, const float* u2c,
                       const float* u2p, const float* u3c, const float* u3p, float beta,
                       float beta_next, const float step[3], const float theta[3],
                       hipStream_t s) {
  const Grid3 G = grid3(P);
  const size_t vol = P->v_elems();
  if (vol == 0) return hipSuccess;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(blocks_for(vol)), dim3(256), 0, s, n1, n2, n3, pq, w, u1c, u1p,
                       u2c, u2p, u3c, u3p, beta, beta_next, step[0], step[1], step[2], theta[0],
                       theta[1], theta[2], P->sw, P->d_phi, P->d_stab_t, G);
  };
  const int ns = P->sw.ns;
  if (ns <= 2) go(r3_u_kernel<2>);
  else if (ns == 3) go(r3_u_kernel<3>);
  else if (ns == 4) go(r3_u_kernel<4>);
  else go(r3_u_kernel<kMaxSpecies>);
  return hipGetLastError();
}

hipError_t launch_tvs_sum(const psoam_plan* P, const float* c, double* partial, double* out,
                          hipStream_t s) {
  const Grid3 G = grid3(P);
  const size_t nb = reduce_blocks((int64_t)P->v_elems());
  hipLaunchKernelGGL(tvs_kernel, dim3((unsigned)nb), dim3(256), 0, s, c, P->sw, P->d_phi,
                     P->d_stab_t, P->Kp, G, partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partial, (int64_t)nb, out,
                     gate_now());
  return hipGetLastError();
}

// ---- per-voxel unmixing (second step of the two-step method) --------------
// g[s][v] = sum_k S_v[k][s] (sum_s' S_v[k][s'] x[s'][v] - b[k][v]) (b may be
// null); with partial, FP64 block sums of sum_k (S x - b)^2
__global__ __launch_bounds__(256) void unmix_grad_kernel(float* __restrict__ g,
                                                         const float* __restrict__ x,
                                                         const float* __restrict__ b,
                                                         SwitchParams sw,
                                                         const float* __restrict__ phi,
                                                         const float* __restrict__ stab, int kp,
                                                         Grid3 G, double* __restrict__ partial) {
  if (G.gate && *G.gate) return;  // a device stop test has ended the solve
  __shared__ double sh[4];
  const int64_t vol = (int64_t)G.ny * G.nx * G.nz;
  double ss = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < vol; v += stride) {
    const int iz = (int)(v % G.nz);
    const size_t col = (size_t)v - iz;
    float xv[kMaxSpecies], acc[kMaxSpecies];
    for (int s = 0; s < sw.ns; ++s) {
      xv[s] = x[(int64_t)s * vol + v];
      acc[s] = 0.0f;
    }
    for (int k = 0; k < sw.nk; ++k) {
      float r = b ? -b[(int64_t)k * vol + v] : 0.0f;
      for (int s = 0; s < sw.ns; ++s) r += coef_zt(sw, phi, stab, G.nz, col, iz, k, s) * xv[s];
      for (int s = 0; s < sw.ns; ++s) acc[s] += coef_zt(sw, phi, stab, G.nz, col, iz, k, s) * r;
      ss += (double)r * (double)r;
    }
    for (int s = 0; s < sw.ns; ++s) g[(int64_t)s * vol + v] = acc[s];
  }
  if (partial) {
    const double r = block_sum(ss, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
  }
}

size_t unmix_blocks(const psoam_plan* P) { return reduce_blocks((int64_t)P->v_elems()); }

hipError_t launch_unmix_grad(const psoam_plan* P, float* g, const float* x, const float* b,
                             double* partial, hipStream_t s) {
  const Grid3 G = grid3(P);
  const size_t nb = partial ? unmix_blocks(P) : blocks_for(P->v_elems());
  hipLaunchKernelGGL(unmix_grad_kernel, dim3((unsigned)nb), dim3(256), 0, s, g, x, b, P->sw,
                     P->d_phi, P->d_stab_t, P->Kp, G, partial);
  return hipGetLastError();
}

// ---- separable switching: pulse expansion and contraction -----------------
struct SepG {
  float g[kMaxSpecies * kMaxSpecies];
};

__global__ __launch_bounds__(256) void sep_expand_kernel(float* __restrict__ y,
                                                         const float* __restrict__ h,
                                                         const float* __restrict__ T, int ns,
                                                         int nk, int64_t n,
                                                         const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float hv[kMaxSpecies];
    for (int s = 0; s < ns; ++s) hv[s] = h[(int64_t)s * n + i];
    for (int k = 0; k < nk; ++k) {
      float acc = 0.0f;
      for (int s = 0; s < ns; ++s) acc += T[k * ns + s] * hv[s];
      y[(int64_t)k * n + i] = acc;
    }
  }
}

__global__ __launch_bounds__(256) void sep_contract_kernel(float* __restrict__ out,
                                                           const float* __restrict__ y,
                                                           const float* __restrict__ T, int ns,
                                                           int nk, int64_t n,
                                                           const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float acc[kMaxSpecies];
    for (int s = 0; s < ns; ++s) acc[s] = 0.0f;
    for (int k = 0; k < nk; ++k) {
      const float v = y[(int64_t)k * n + i];
      for (int s = 0; s < ns; ++s) acc[s] += T[k * ns + s] * v;
    }
    for (int s = 0; s < ns; ++s) out[(int64_t)s * n + i] = acc[s];
  }
}

__global__ __launch_bounds__(256) void sep_residual_kernel(float* __restrict__ rt,
                                                           const float* __restrict__ h,
                                                           const float* __restrict__ q, SepG G,
                                                           int ns, int64_t n,
                                                           double* __restrict__ partial,
                                                           const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  __shared__ double sh[4];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float hv[kMaxSpecies];
    for (int s = 0; s < ns; ++s) hv[s] = h[(int64_t)s * n + i];
    for (int s = 0; s < ns; ++s) {
      float r = 0.0f;
      for (int t = 0; t < ns; ++t) r += G.g[s * kMaxSpecies + t] * hv[t];
      const float qv = q ? q[(int64_t)s * n + i] : 0.0f;
      r -= qv;
      rt[(int64_t)s * n + i] = r;
      acc += (double)hv[s] * ((double)r - (double)qv);
    }
  }
  if (partial) {
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
  }
}

// Temporal convolution pass of the factorised operator (eq.
// acoustic-temporal-conv on every A-scan): one wave per row of nt samples,
// staged in LDS with kMaxEir zero samples on either side so that every tap
// reads inside the buffer; modes 2 and 3 put the residual in a second row
// buffer.  The grid strides over groups of rows; every wave of a block runs
// the same number of groups (block-uniform loop), so the barriers match.
//   mode 0: out[t] = sum_j v[j] in[t - j + origin]
//   mode 1: out[t] = sum_j v[j] in[t + j - origin]          (the adjoint)
//   mode 2: r = (V in) - p, out = V^T r, FP64 block sums of r^2
//   mode 3: r = (V in) - p, FP64 block sums of r^2 only
// `out` may alias `in` (each row is read whole before it is written).
template <int MODE, bool VEC>
__global__ __launch_bounds__(256) void eir_rows_kernel(float* out, const float* in,
                                                       const float* __restrict__ pm, EirParams e,
                                                       int nt, int64_t rows,
                                                       double* __restrict__ partial) {
  if (e.gate && *e.gate) return;  // a device stop test has ended the solve
  extern __shared__ float eir_lds[];
  __shared__ double sh[4];
  const int wpb = (int)(blockDim.x >> 6), w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int stride = nt + 2 * kMaxEir;
  float* qb = eir_lds + (size_t)w * stride * (MODE >= 2 ? 2 : 1);
  float* rb = qb + stride;
  // VEC (nt a multiple of 4, 16-byte aligned rows): a lane moves and computes
  // 4 consecutive samples; the row buffers stay 16-byte aligned (kMaxEir and
  // stride are multiples of 4)
  constexpr int E = VEC ? 4 : 1;
  const int nv = nt / E;
  double ss = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * wpb; base < rows; base += (int64_t)gridDim.x * wpb) {
    const int64_t row = base + w;
    const bool live = row < rows;
    const size_t off = live ? (size_t)row * nt : 0;
    if constexpr (VEC) {
      for (int i = lane; i < nv; i += 64) {
        const f32x4 v = live ? *(const f32x4*)(in + off + 4 * i) : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        *(f32x4*)(qb + kMaxEir + 4 * i) = v;
      }
      for (int i = lane; i < kMaxEir; i += 64) {
        qb[i] = 0.0f;
        qb[kMaxEir + nt + i] = 0.0f;
        if (MODE >= 2) {
          rb[i] = 0.0f;
          rb[kMaxEir + nt + i] = 0.0f;
        }
      }
    } else {
      for (int i = lane; i < stride; i += 64) {
        const int t = i - kMaxEir;
        qb[i] = (live && t >= 0 && t < nt) ? in[off + t] : 0.0f;
        if (MODE >= 2 && (t < 0 || t >= nt)) rb[i] = 0.0f;
      }
    }
    __syncthreads();
    if (MODE <= 1) {
      for (int i = lane; i < nv; i += 64) {
        float acc[E];
#pragma unroll
        for (int u = 0; u < E; ++u) acc[u] = 0.0f;
        for (int j = 0; j < e.n; ++j) {
          const int lag = j - e.origin;
          const float* src = qb + kMaxEir + E * i + (MODE == 0 ? -lag : lag);
#pragma unroll
          for (int u = 0; u < E; ++u) acc[u] += e.v[j] * src[u];
        }
        if (live) {
          if constexpr (VEC) *(f32x4*)(out + off + 4 * i) = f32x4{acc[0], acc[1], acc[2], acc[3]};
          else out[off + i] = acc[0];
        }
      }
    } else {
      for (int i = lane; i < nv; i += 64) {
        float acc[E];
#pragma unroll
        for (int u = 0; u < E; ++u) acc[u] = 0.0f;
        for (int j = 0; j < e.n; ++j) {
          const float* src = qb + kMaxEir + E * i - (j - e.origin);
#pragma unroll
          for (int u = 0; u < E; ++u) acc[u] += e.v[j] * src[u];
        }
        float pv[E];
        if constexpr (VEC) {
          const f32x4 q4 = (pm && live) ? *(const f32x4*)(pm + off + 4 * i) : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int u = 0; u < E; ++u) pv[u] = q4[u];
        } else {
          pv[0] = (pm && live) ? pm[off + i] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < E; ++u) {
          const float r = acc[u] - pv[u];
          rb[kMaxEir + E * i + u] = r;
          if (live) ss += (double)r * (double)r;
        }
      }
      if (MODE == 2) {
        __syncthreads();
        for (int i = lane; i < nv; i += 64) {
          float acc[E];
#pragma unroll
          for (int u = 0; u < E; ++u) acc[u] = 0.0f;
          for (int j = 0; j < e.n; ++j) {
            const float* src = rb + kMaxEir + E * i + (j - e.origin);
#pragma unroll
            for (int u = 0; u < E; ++u) acc[u] += e.v[j] * src[u];
          }
          if (live) {
            if constexpr (VEC) *(f32x4*)(out + off + 4 * i) = f32x4{acc[0], acc[1], acc[2], acc[3]};
            else out[off + i] = acc[0];
          }
        }
      }
    }
    __syncthreads();  // the next group overwrites the row buffers
  }
  if (MODE >= 2 && partial) {
    const double r = block_sum(ss, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
  }
}

static inline int eir_waves(int nt) { return nt <= 1024 ? 4 : 1; }

size_t eir_blocks(const psoam_plan* P) {
  const int64_t rows = (int64_t)P->g.n_pulses * P->g.ny * P->g.nx;
  const int wpb = eir_waves(P->g.nt);
  const int64_t b = (rows + wpb - 1) / wpb;
  return (size_t)std::min<int64_t>(std::max<int64_t>(b, 1), 2048);
}

hipError_t launch_eir_rows(const psoam_plan* P, int mode, float* out, const float* in,
                           const float* p, double* partial, hipStream_t s) {
  const int nt = P->g.nt;
  if (nt <= 0 || nt > kMaxEirNt) return hipErrorInvalidValue;
  const int64_t rows = (int64_t)P->g.n_pulses * P->g.ny * P->g.nx;
  if (rows == 0) return hipSuccess;
  const int wpb = eir_waves(nt);
  const size_t lds = sizeof(float) * (size_t)wpb * (nt + 2 * kMaxEir) * (mode >= 2 ? 2 : 1);
  const dim3 grid((unsigned)eir_blocks(P)), block(64 * wpb);
  auto al16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
  const bool vec = (nt & 3) == 0 && al16(out) && al16(in) && al16(p);
  EirParams ep = P->eir;
  ep.gate = gate_now();
#define PSOAM_EIR(M)                                                                        \
  {                                                                                         \
    if (vec)                                                                                \
      hipLaunchKernelGGL((eir_rows_kernel<M, true>), grid, block, lds, s, out, in, p, ep, nt, \
                         rows, partial);                                                    \
    else                                                                                    \
      hipLaunchKernelGGL((eir_rows_kernel<M, false>), grid, block, lds, s, out, in, p, ep, nt, \
                         rows, partial);                                                    \
    break;                                                                                  \
  }
  switch (mode) {
    case 0: PSOAM_EIR(0)
    case 1: PSOAM_EIR(1)
    case 2: PSOAM_EIR(2)
    case 3: PSOAM_EIR(3)
    default:
      return hipErrorInvalidValue;
  }
#undef PSOAM_EIR
  return hipGetLastError();
}

// The factorised H^T operand in one pass: the temporal pass (eq.
// acoustic-temporal-conv) and its adjoint fused with the rounding and
// packing of the 16-bit octet operand rq[pos][t/8][k][8] (pack_r16's layout,
// samples shifted by tsh).  A block takes the 16 pulses kc..kc+15 of one scan
// position; their rows sit in LDS between zero margins (kEirL samples
// before, kEirR after, which cover every tap of every sample the block
// reads; the row stride is odd so the 16 rows fall in different banks).
//   RESID: r = V q - p (p may be null), then V^T r;  otherwise V^T q.
// A thread makes 8 consecutive samples from a register window that slides
// one sample per tap (one LDS read per tap instead of eight); the taps are
// summed in the order eir_rows_kernel sums them.  The octet of (octet o,
// pulse a) goes straight to HBM: 16 consecutive threads write the 256
// contiguous bytes of one octet's 16 pulses.
constexpr int kEirL = 40, kEirR = 64;
constexpr size_t kEirPackMaxLds = 128 * 1024;
__host__ __device__ inline int eir_pack_stride(int nt) { return (nt + kEirL + kEirR) | 1; }
// the residual form holds two row buffers (46 KB at Nt 256, three blocks per
// CU), so it runs 8 waves per block to keep 24 waves on a CU, as the
// one-buffer form does with 4
__host__ __device__ constexpr int eir_pack_threads(bool resid) { return resid ? 512 : 256; }

template <int PREC, bool SPLIT, bool RESID>
__global__ __launch_bounds__(512) void eir_pack16(const float* __restrict__ q,
                                                  const float* __restrict__ pm, EirParams e,
                                                  typename Half<PREC>::E* __restrict__ rq,
                                                  typename Half<PREC>::E* __restrict__ rq_lo,
                                                  int nk, int ny, int nx, int nt, int to_n,
                                                  int kp, int xp, int r, size_t ps, int tsh,
                                                  const float* __restrict__ f16) {
  if (e.gate && *e.gate) return;  // a device stop test has ended the solve
  using H = Half<PREC>;
  using V = typename H::V;
  const float sc = f16 ? f16[2] : H::scale;   // operand scale (FP16: per call)
  constexpr int NTH = eir_pack_threads(RESID);
  extern __shared__ float ep_lds[];
  const int sst = eir_pack_stride(nt);
  float* qb = ep_lds;
  float* rb = ep_lds + 16 * sst;
  const int groups = kp / 16;
  const int pos = (int)(blockIdx.x / groups);
  const int kc = (int)(blockIdx.x % groups) * 16;
  const int y = pos / nx, x = pos - y * nx;
  const int tid = (int)threadIdx.x;
  const size_t plane = (size_t)ny * nx * nt;              // pulse stride of the A-scans
  const size_t col = ((size_t)y * nx + x) * nt;           // this position's row in a pulse
  // residual units (8 samples of one row) and the measurements of this
  // thread's first kEirPre units, loaded now so that their latency overlaps
  // the staging of the rows
  const int nu = (nt + 7) >> 3;
  auto load_p = [&](int i, float (&p8)[8]) {
    const int a = i / nu, t0 = (i - a * nu) * 8;
    const int k = kc + a;
    const bool live = pm && i < 16 * nu && k < nk;
    const float* prow = live ? pm + (size_t)k * plane + col + t0 : pm;
#pragma unroll
    for (int u = 0; u < 8; ++u) p8[u] = (live && t0 + u < nt) ? prow[u] : 0.0f;
  };
  constexpr int kEirPre = 2;
  float pre[kEirPre][8];
  if constexpr (RESID) {
#pragma unroll
    for (int m = 0; m < kEirPre; ++m) load_p(tid + m * NTH, pre[m]);
  }
  // zero margins: columns [0, kEirL) and [kEirL + nt, sst) of every row
  const int padn = sst - nt;
  for (int i = tid; i < 16 * padn; i += NTH) {
    const int a = i / padn, m = i - a * padn;
    const int cc = a * sst + (m < kEirL ? m : nt + m);
    qb[cc] = 0.0f;
    if constexpr (RESID) rb[cc] = 0.0f;
  }
  // the rows, kEirBatch loads in flight per thread before any LDS write
  constexpr int kEirBatch = 8;
  const int nin = 16 * nt;
  for (int base = 0; base < nin; base += NTH * kEirBatch) {
    float v[kEirBatch];
#pragma unroll
    for (int b = 0; b < kEirBatch; ++b) {
      const int i = base + b * NTH + tid;
      const int a = i / nt, t = i - a * nt;
      v[b] = (i < nin && kc + a < nk) ? q[(size_t)(kc + a) * plane + col + t] : 0.0f;
    }
#pragma unroll
    for (int b = 0; b < kEirBatch; ++b) {
      const int i = base + b * NTH + tid;
      const int a = i / nt, t = i - a * nt;
      if (i < nin) qb[a * sst + kEirL + t] = v[b];
    }
  }
  __syncthreads();
  if constexpr (RESID) {
    auto unit = [&](int i, const float (&pv)[8]) {
      const int a = i / nu, t0 = (i - a * nu) * 8;
      // src[u - j] = q[t0 + u - j + origin]
      const float* src = qb + a * sst + kEirL + t0 + e.origin;
      float w[8], acc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        w[u] = src[u];
        acc[u] = 0.0f;
      }
      for (int j = 0; j < e.n; ++j) {
        if (j > 0) {
#pragma unroll
          for (int u = 7; u > 0; --u) w[u] = w[u - 1];
          w[0] = src[-j];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += e.v[j] * w[u];
      }
      float* dst = rb + a * sst + kEirL + t0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (t0 + u < nt) dst[u] = acc[u] - pv[u];
    };
    int i = tid;
#pragma unroll
    for (int m = 0; m < kEirPre; ++m, i += NTH)
      if (i < 16 * nu) unit(i, pre[m]);
    for (; i < 16 * nu; i += NTH) {
      float pv[8];
      load_p(i, pv);
      unit(i, pv);
    }
    __syncthreads();
  }
  const float* sb = RESID ? rb : qb;
  const size_t o_pos = ((size_t)(y + r) * xp + (x + r)) * ps;
  for (int i = tid; i < 16 * to_n; i += NTH) {
    const int o = i >> 4, a = i & 15;
    const int t0 = o * 8 - tsh;
    // src[u + j] = r[t0 + u + j - origin]
    const float* src = sb + a * sst + kEirL + t0 - e.origin;
    float w[8], acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      w[u] = src[u];
      acc[u] = 0.0f;
    }
    for (int j = 0; j < e.n; ++j) {
      if (j > 0) {
#pragma unroll
        for (int u = 0; u < 7; ++u) w[u] = w[u + 1];
        w[7] = src[7 + j];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += e.v[j] * w[u];
    }
    V hi, lo;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float v = (t0 + u >= 0 && t0 + u < nt) ? acc[u] * sc : 0.0f;
      hi[u] = (typename H::E)v;
      lo[u] = (typename H::E)(v - (float)hi[u]);
    }
    const size_t off = o_pos + ((size_t)o * kp + kc + a) * 8;
    *(V*)(rq + off) = hi;
    if constexpr (SPLIT) *(V*)(rq_lo + off) = lo;
  }
}

static size_t eir_pack_lds(const psoam_plan* P, bool resid) {
  return sizeof(float) * 16 * (size_t)eir_pack_stride(P->g.nt) * (resid ? 2 : 1);
}

bool eir_pack_fits(const psoam_plan* P, bool resid) {
  if (!P->fact || P->prec == PSOAM_FP32) return false;
  // PSOAM_EIR_PACK=0 keeps the two-pass form (row pass, then pack_r16)
  if (const char* ev = std::getenv("PSOAM_EIR_PACK"))
    if (ev[0] == '0') return false;
  return P->g.nt <= kMaxEirNt && eir_pack_lds(P, resid) <= kEirPackMaxLds;
}

hipError_t launch_eir_pack(const psoam_plan* P, const float* q, const float* p, bool resid,
                           hipStream_t s) {
  if (!eir_pack_fits(P, resid)) return hipErrorInvalidValue;
  EirParams ep = P->eir;
  ep.gate = gate_now();
  if (P->d_f16) {
    // V^T (V q - p) with q = Lambda S x: bound l1 (l1 hrow srow max|x| + max|p|),
    // l1 = sum |v|; the adjoint's V^T y: l1 max|y|
    const double l1 = P->eir_l1;
    hipError_t e = hipSuccess;
    if (resid) {
      e = f16_scale(P, 3, l1 * l1 * P->hrow * P->srow, l1, s);
    } else {
      e = f16_amax(P, q, (int64_t)P->y_elems(), 1, s);
      if (e == hipSuccess) e = f16_scale(P, 1, l1, 0.0, s);
    }
    if (e != hipSuccess) return e;
  }
  const auto& g = P->g;
  const size_t lds = eir_pack_lds(P, resid);
  const size_t nb = (size_t)g.ny * g.nx * (P->Kp / 16);
  if (nb == 0) return hipSuccess;
#define PSOAM_EP_R(PR, SP, RS)                                                              \
  {                                                                                         \
    using E = Half<PR>::E;                                                                  \
    auto kern = eir_pack16<PR, SP, RS>;                                                     \
    if (lds > 64 * 1024)                                                                    \
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                (int)lds);                                                  \
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(eir_pack_threads(RS)), lds, s, q, p, \
                       ep,                                                                  \
                       (E*)P->d_rq, (E*)P->d_rq_lo, g.n_pulses, g.ny, g.nx, g.nt, P->Lt / 8, \
                       P->Kp, P->Xp, P->R, P->ps_r, P->tsh, P->d_f16);                      \
  }
#define PSOAM_EP(PR, SP)                                                                    \
  {                                                                                         \
    if (resid) PSOAM_EP_R(PR, SP, true) else PSOAM_EP_R(PR, SP, false)                      \
    break;                                                                                  \
  }
  switch (P->prec) {
    case PSOAM_BF16:
    case PSOAM_BF16_REFINED: PSOAM_EP(PSOAM_BF16, false)
    case PSOAM_FP16: PSOAM_EP(PSOAM_FP16, false)
    case PSOAM_BF16_SPLIT: PSOAM_EP(PSOAM_BF16, true)
    case PSOAM_FP16_SPLIT: PSOAM_EP(PSOAM_FP16, true)
    default:
      return hipErrorInvalidValue;
  }
#undef PSOAM_EP
#undef PSOAM_EP_R
  return hipGetLastError();
}

size_t sep_blocks(const psoam_plan* P) {
  return reduce_blocks((int64_t)((size_t)P->g.ny * P->g.nx * P->g.nt));
}

hipError_t launch_sep_expand(const psoam_plan* P, float* y, const float* h, hipStream_t s) {
  const int64_t n = (int64_t)P->g.ny * P->g.nx * P->g.nt;
  hipLaunchKernelGGL(sep_expand_kernel, dim3(blocks_for((size_t)n)), dim3(256), 0, s, y, h,
                     (const float*)P->d_T, P->g.n_species, P->g.n_pulses, n, gate_now());
  return hipGetLastError();
}

hipError_t launch_sep_contract(const psoam_plan* P, float* out, const float* y, hipStream_t s) {
  const int64_t n = (int64_t)P->g.ny * P->g.nx * P->g.nt;
  hipLaunchKernelGGL(sep_contract_kernel, dim3(blocks_for((size_t)n)), dim3(256), 0, s, out, y,
                     (const float*)P->d_T, P->g.n_species, P->g.n_pulses, n, gate_now());
  return hipGetLastError();
}

hipError_t launch_sep_residual(const psoam_plan* P, float* rt, const float* h, const float* q,
                               double* partial, hipStream_t s) {
  const int64_t n = (int64_t)P->g.ny * P->g.nx * P->g.nt;
  SepG G;
  for (int i = 0; i < kMaxSpecies * kMaxSpecies; ++i) G.g[i] = P->sep_g[i];
  const size_t nb = partial ? sep_blocks(P) : blocks_for((size_t)n);
  hipLaunchKernelGGL(sep_residual_kernel, dim3((unsigned)nb), dim3(256), 0, s, rt, h, q, G,
                     P->g.n_species, n, partial, gate_now());
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void scale_rnorm_kernel(float* __restrict__ v,
                                                          const float* __restrict__ w,
                                                          const double* __restrict__ norm2,
                                                          int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double inv = 1.0 / sqrt(norm2[0]);
  v[i] = (float)((double)w[i] * inv);
}

hipError_t launch_scale_by_rnorm(float* v, const float* w, const double* norm2, int64_t n,
                                 hipStream_t s) {
  hipLaunchKernelGGL(scale_rnorm_kernel, dim3(blocks_for((size_t)n)), dim3(256), 0, s, v, w,
                     norm2, n);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void momentum_kernel(float* __restrict__ xi,
                                                       const float* __restrict__ cn,
                                                       const float* __restrict__ cp, float beta,
                                                       int64_t n, double* __restrict__ partial,
                                                       const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  __shared__ double sh[4];
  double dd = 0.0, nn = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float a = cn[i];
    const float xn = a + beta * (a - cp[i]);
    const float xo = xi[i];
    dd += ((double)xn - (double)xo) * ((double)xn - (double)xo);
    nn += (double)xo * (double)xo;
    xi[i] = xn;
  }
  const double r0 = block_sum(dd, sh);
  const double r1 = block_sum(nn, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = r0;
    partial[gridDim.x + blockIdx.x] = r1;
  }
}

hipError_t launch_momentum(float* xi, const float* c_next, const float* c_prev, float beta,
                           int64_t n, double* partial, hipStream_t s) {
  const size_t nb = reduce_blocks(n);
  hipLaunchKernelGGL(momentum_kernel, dim3((unsigned)nb), dim3(256), 0, s, xi, c_next, c_prev,
                     beta, n, partial, gate_now());
  return hipGetLastError();
}

// Momentum with the FISTA step state on the device (for captured iterations,
// whose kernel arguments are fixed): t_k is read from tst[0], the weight is
// formed in FP64 exactly as the host does (Beck-Teboulle (t-1)/t', or the
// printed (t-1)/(t+1)), and xi = c_{k+1} + beta (c_{k+1} - c_k).
__global__ __launch_bounds__(256) void momentum_dev_kernel(float* __restrict__ xi,
                                                           const float* __restrict__ cn,
                                                           const float* __restrict__ cp,
                                                           const double* __restrict__ tst,
                                                           int literal, int64_t n,
                                                           double* __restrict__ partial,
                                                           const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  __shared__ double sh[4];
  const double t = tst[0];
  const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
  const float beta = (float)(literal ? (t - 1.0) / (t + 1.0) : (t - 1.0) / tn);
  double dd = 0.0, nn = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float a = cn[i];
    const float xn = a + beta * (a - cp[i]);
    if (partial) {
      // the same partial sums as momentum_kernel (for the xi-change test)
      const float xo = xi[i];
      dd += ((double)xn - (double)xo) * ((double)xn - (double)xo);
      nn += (double)xo * (double)xo;
    }
    xi[i] = xn;
  }
  if (partial) {
    const double r0 = block_sum(dd, sh);
    const double r1 = block_sum(nn, sh);
    if (threadIdx.x == 0) {
      partial[blockIdx.x] = r0;
      partial[gridDim.x + blockIdx.x] = r1;
    }
  }
}

// t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, one thread, after the momentum kernel
__global__ void advance_t_kernel(double* tst, const int* __restrict__ gate) {
  if (gate && *gate) return;  // a device stop test has ended the solve
  const double t = tst[0];
  tst[0] = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
}

__global__ void set_double_kernel(double* p, double v) { p[0] = v; }

// ---- device-side stopping tests (Alg. alg:prox-outer, both tests) ----------
// ctl: [0] stopped, [1] iterations done, [2] objective not finite,
//      [3] index of the next iteration;
// sc (the plan's FP64 scalars): [2], [3] |xi_{k+1} - xi_k|^2 and |xi_k|^2,
//      [4..7] data term, TV, l1, TV(S c) of c_{k+1}, [9] |p|^2 (separable),
//      [10] previous objective, [11] 1 once there is one, [12] last objective
__global__ void stop_init_kernel(int* ctl, double* sc) {
  ctl[0] = ctl[1] = ctl[2] = ctl[3] = 0;
  sc[10] = 0.0;
  sc[11] = 0.0;
  sc[12] = __builtin_nan("");
}

// One thread, after iteration k's momentum and objective terms: the same
// decisions as the host-side tests, in the same FP64 arithmetic.
__global__ void stop_test_kernel(int* ctl, double* sc, double* trace, StopTest t) {
  // no fused multiply-adds: every operation rounds as on the host
#pragma clang fp contract(off)
  if (ctl[0]) return;
  const int k = ctl[3];
  ctl[3] = k + 1;
  ctl[1] = k + 1;
  double f_now = 0.0;
  if (t.need_obj) {
    const double data = t.add_p2 ? sc[4] + sc[9] : sc[4];
    f_now = 0.5 * data + t.lam_tv * sc[5] + t.lam_l1 * sc[6];
    if (t.tvs) f_now += t.lam_tvs * sc[7];
    if (!isfinite(f_now)) {
      ctl[2] = 1;
      ctl[0] = 1;
      return;
    }
    if (trace) trace[k] = f_now;
    sc[12] = f_now;
  }
  bool stop = false;
  if (k > 1) {
    if (t.eps1 > 0.0 && sc[11] != 0.0 && fabs(f_now - sc[10]) < t.eps1 * fabs(sc[10])) stop = true;
    if (t.eps2 > 0.0 && sc[3] > 0.0 && sqrt(sc[2]) < t.eps2 * sqrt(sc[3])) stop = true;
  }
  if (t.need_obj) {
    sc[10] = f_now;
    sc[11] = 1.0;
  }
  if (stop) ctl[0] = 1;
}

// out = the buffer holding the last iterate: iteration k writes c_{k+1} into
// the buffer that was "next" at k, which alternates, so after n iterations it
// is a1 for odd n and a0 for even n
__global__ __launch_bounds__(256) void select_copy_kernel(float* __restrict__ out,
                                                          const float* __restrict__ a0,
                                                          const float* __restrict__ a1,
                                                          const int* __restrict__ ctl, int64_t n) {
  const float* src = (ctl[1] & 1) ? a1 : a0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = src[i];
}

hipError_t launch_stop_init(int* ctl, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(stop_init_kernel, dim3(1), dim3(1), 0, s, ctl, sc);
  return hipGetLastError();
}

hipError_t launch_stop_test(int* ctl, double* sc, double* trace, const StopTest& t, hipStream_t s) {
  hipLaunchKernelGGL(stop_test_kernel, dim3(1), dim3(1), 0, s, ctl, sc, trace, t);
  return hipGetLastError();
}

hipError_t launch_select_copy(float* out, const float* a0, const float* a1, const int* ctl,
                              int64_t n, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<size_t>(blocks_for((size_t)n), 4096);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(select_copy_kernel, dim3(nb), dim3(256), 0, s, out, a0, a1, ctl, n);
  return hipGetLastError();
}

hipError_t launch_momentum_dev(float* xi, const float* c_next, const float* c_prev, double* tst,
                               int literal, int64_t n, double* partial, hipStream_t s) {
  const size_t nb = reduce_blocks(n);
  hipLaunchKernelGGL(momentum_dev_kernel, dim3((unsigned)nb), dim3(256), 0, s, xi, c_next, c_prev,
                     (const double*)tst, literal, n, partial, gate_now());
  hipLaunchKernelGGL(advance_t_kernel, dim3(1), dim3(1), 0, s, tst, gate_now());
  return hipGetLastError();
}

hipError_t launch_set_double(double* p, double v, hipStream_t s) {
  hipLaunchKernelGGL(set_double_kernel, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

}  // namespace psoam
