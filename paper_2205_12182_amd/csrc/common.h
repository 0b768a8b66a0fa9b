// Internal definitions shared by the NOLSM HIP kernels (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <vector>

#include "nolsm.h"

namespace nolsm {

// Submatrix dimensions are padded to a multiple of PAD.  The padding of T_k(S)
// is the identity and the padding of T_k(H0) is zero, so the padded matrices
// factor as diag(L, I) and every padded iterate stays zero outside the n x n
// block.
constexpr int PAD = 64;
constexpr int NB = 64;             // FP64 Cholesky / inverse block size
constexpr int ST = 128;            // sign-iteration output tile (ST x ST)
constexpr int RESID_SHIFT = 40;    // fixed-point scale of the residual accumulator
constexpr float RESID_CLAMP = 1.0e4f;
constexpr int NPANEL = 8;         // n x m FP32 panel slots per submatrix
constexpr int MAXM = 32;          // own columns per panel-kernel workgroup (column chunk)
constexpr int MAX_OWN = 8192;     // own columns of a submatrix (chunks of MAXM columns)
constexpr int ENERGY_NOALLOC_MAXMOL = NOLSM_ENERGY_NOALLOC_MAXMOL;   // nolsm_energy_noalloc limit
constexpr int MAX_DEVICES = 64;   // devices whose scratch address is cached

enum Prec : int32_t { P_FP32 = 0, P_FP16 = 1, P_BF16 = 2 };

// Per-submatrix description (device, read-only after bind).  A submatrix serves the
// block columns of ngrp molecules (one, or a combined group): members own_mem ..
// own_mem + ngrp - 1 of its member list, whose functions are its own columns
// own_lo .. own_lo + m - 1.
struct SubDesc {
  int32_t n, npad, mol, m;          // dimension, leading dimension, first own molecule, own columns
  int32_t own_lo, nmem, mem_off, ngrp;
  int32_t own_mem, kb;              // kb: the FP16/BF16 iterate is k-blocked (kb_index)
  int64_t off_h;                    // bytes from workspace base: FP64 npad^2 H_k, then FP32 M_k
  int64_t off_s;                    // FP64 npad^2 (S_k -> L -> L^-1)
  int64_t off_lo;                   // 3 x (4 npad^2) bytes: sign-iteration buffers / FP64 scratch
  int64_t off_diag;                 // FP64 2 x npad x NB: inverted diagonal blocks + panel temp
  int64_t off_panel;                // FP32 NPANEL x npad x m panels
  int64_t off_dcol;                 // FP64 npad x m density columns
};

// Per-submatrix mutable state (device).
struct SubState {
  double scale;                     // b_k
  double lower;                     // current lower bound l on |eig(X)| (scaled iteration)
  unsigned long long racc;          // fixed-point sum of (X^2 - I)^2
  unsigned long long scale_bits;    // Gershgorin max as ordered bits (positive doubles)
  float resid;                      // last ||X^2 - I||_F
  int32_t status;                   // 0, NOLSM_ENOTSPD, NOLSM_ENOCONV
  int32_t active;                   // iterating in the current phase
  int32_t cur;                      // buffer (0..2) holding the current X
  int32_t prec;                     // precision of the buffers (Prec)
  int32_t iters_lo, iters_fb, fell_back;
  int32_t extra_left;               // iterations still to run after reaching tol (-1: not reached)
  int32_t converged;
  float c1, c3;                     // coefficients of the next update X <- c1 X + c3 X Y
  float tr_x;                       // Tr(X) of the final iterate
  float pad_;
};

struct Tile { int32_t sub, ti, tj, pad; };

// k-blocked layout of the sign iterate of submatrices on the 256 x 128 tiles (FP16 and
// BF16): element (row r, column c) at ((r / 32) npad + c) 32 + r % 32, so a 32-row
// chunk of a column is one 64-byte run and the chunks of consecutive columns are
// adjacent.  The products read both factors as column panels 32 k deep, so a stage of
// 256 columns is one contiguous 16 KiB block (instead of 256 runs of 64 bytes one
// column apart).  The cast forms the iterate k-blocked, precision changes keep it (an
// FP32 iterate, on 128 x 128 tiles, is column major), and the panel and trace kernels
// read it in place.
__host__ __device__ __forceinline__ int64_t kb_index(int r, int c, int ld) {
  return ((int64_t)(r >> 5) * ld + c) * 32 + (r & 31);
}

// Tile lists: upper-triangle tiles of the symmetric products, t[0] the small
// submatrices in 128 x 128 tiles, t[1] the large ones in 256 x 128 tiles (FP16 and
// BF16, two workgroups per CU), t[2] the large ones in 128 x 128 tiles (FP32);
// t[3] every 128 x 128 tile of every submatrix (the non-symmetric FP32 set-up
// product); t[4] every 256 x 128 tile and t[5] the upper-triangle 256 x 128 tiles of
// every submatrix (the split-FP16 set-up products).
constexpr int NTILELIST = 6;
struct TileSet {
  const Tile *t[NTILELIST];
  int n[NTILELIST];
  unsigned long long *flop_units;   // executed MFMA work of active tiles, in FLOP_UNIT
  unsigned *fb_count;               // submatrices selected for the FP32 restart
  unsigned *fb_live;                // of those, the ones still iterating (gates its products)
};
// 2 * 16 * 16 * 64 flops: one 16 x 16 output block over 64 k (tile edges and npad
// are multiples of these, so the count is exact)
constexpr double FLOP_UNIT = 32768.0;
constexpr int BIG_TILE_MIN_NPAD = 768;   // submatrices at least this large use 256 x 128 tiles

// Host-side record of HIP event pairs around launch groups (measurement only).
enum TimeCat { T_GATHER = 0, T_SETUP, T_SIGN, T_GEMM, T_PANEL, T_SCATTER, T_NCAT };

struct EventLog {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec { int cat; hipEvent_t a, b; };
  std::vector<Rec> recs;
  int64_t n_gemm = 0;
  double gemm_flop = 0.0;
  double ms[T_NCAT] = {0, 0, 0, 0, 0, 0};

  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      pool.push_back(e);
    }
    return pool[used++];
  }
  int begin(int cat, hipStream_t s) {
    if (!on) return -1;
    Rec r{cat, next(), next()};
    (void)hipEventRecord(r.a, s);
    recs.push_back(r);
    return (int)recs.size() - 1;
  }
  void end(int idx, hipStream_t s) {
    if (idx >= 0) (void)hipEventRecord(recs[idx].b, s);
  }
  // Fold completed records into ms[] (waits for the events), recycle the pool.
  void collect() {
    for (const Rec &r : recs) {
      (void)hipEventSynchronize(r.b);
      float t = 0.0f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) ms[r.cat] += t;
    }
    recs.clear();
    used = 0;
  }
  ~EventLog() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// ------------------------------------------------------------------ small helpers

template <typename T> __device__ __forceinline__ float to_f32(T v);
template <> __device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_f32<_Float16>(_Float16 v) { return (float)v; }
template <> __device__ __forceinline__ float to_f32<__bf16>(__bf16 v) { return (float)v; }

template <typename T> __device__ __forceinline__ T from_f32(float v);
template <> __device__ __forceinline__ float from_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ _Float16 from_f32<_Float16>(float v) { return (_Float16)v; }
template <> __device__ __forceinline__ __bf16 from_f32<__bf16>(float v) { return (__bf16)v; }

template <typename T> __device__ __forceinline__ T from_f64(double v);
template <> __device__ __forceinline__ float from_f64<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ _Float16 from_f64<_Float16>(double v) { return (_Float16)(float)v; }
template <> __device__ __forceinline__ __bf16 from_f64<__bf16>(double v) { return (__bf16)(float)v; }

__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum in a fixed order (deterministic); blockDim.x == 256.
template <typename T>
__device__ __forceinline__ T block_sum256(T v, T *red /* LDS [4] */) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  T r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ unsigned long long resid_fixed(float partial) {
  if (!(partial <= RESID_CLAMP)) partial = RESID_CLAMP;    // also catches NaN
  return (unsigned long long)((double)partial * (double)(1ull << RESID_SHIFT) + 0.5);
}

// Map a flat workgroup id onto a logical tile id so that consecutive logical
// tiles (the tiles of one submatrix) land on the same XCD: workgroups are
// dispatched round-robin over the 8 XCDs, so XCD x runs ids b with b % 8 == x.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

}  // namespace nolsm
