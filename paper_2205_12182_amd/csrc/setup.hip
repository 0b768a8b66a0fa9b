// Set-up of the sign argument for Eq. 8 (FP64 factorisation, FP32 products).
//
// T_k(S)^-1 T_k(H0) - mu I has the same spectrum as the symmetric matrix
//   M_k - mu I,  M_k = L^-1 T_k(H0) L^-T,  T_k(S) = L L^T,
// and sign(S^-1 H - mu I) = L^-T sign(M - mu I) L^T, so Eq. 8 becomes
//   T_k(D) = 1/2 L^-T (I - sign(M_k - mu I)) L^-1.
// M_k does not depend on mu; mu is applied when the first iterate is formed.
//
// Kernels (all batched over the planned submatrices, one launch per block step):
//   chol_diag    unblocked Cholesky of a 64x64 diagonal block in LDS, plus its inverse
//   chol_panel   A[j+64:, j] <- A[j+64:, j] L_jj^-T                  (FP64 MFMA)
//   chol_update, chol_update128, chol_trail
//                A[j+64:, j+64:] -= P P^T, lower tiles: left-looking inside an outer
//                block, right-looking between blocks (FP32 MFMA tiles on an FP32 copy
//                of the panel; FP64 MFMA as a plan option)
//   trtri_*      L^-1 in place, block columns right to left (outer products on FP32
//                MFMA tiles, the rest FP64 MFMA)
//   prep_split     L^-1 and H split into FP16 pairs (x = hi + 2^-11 lo), by rows
//   split_gemm     U = H L^-T, then M = L^-1 U, upper tiles mirrored so that M is
//                  exactly symmetric; M is kept in FP32 over the H buffer (FP16 MFMA,
//                  three partial products per term, FP32 sums)
//   prep_products / setup_gemm   the same two products on FP32 operands and FP32
//                  MFMAs (plan option)
// M only feeds the low-precision sign iteration and its scaling; the density
// columns use the FP64 L^-1, so the rounding in M (relative ~1e-7 with FP32
// operands, a few 1e-7 with split FP16 operands) stays far below the FP16
// rounding of the iteration.
#include <type_traits>

#include "common.h"
#include "ns_gemm.h"
#include "ns_gemm_split.h"

namespace nolsm {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int KS64 = 16;           // k per LDS stage
constexpr int LDP = 64 + 1;        // padded LDS row (doubles)

// acc += A[i0:i0+64, k0:k1] * opB(B)[k0:k1, j0:j0+64]   (A column major, lda)
// TRANSB = false: B(k, n) at B[n * ldb + k];  true: B(k, n) at B[k * ldb + n].
// Wave w owns rows (w >> 1) * 32, cols (w & 1) * 32 as 2 x 2 blocks of 16 x 16.
// v_mfma_f64_16x16x4_f64 takes A(i, k) from lane i + 16 k and B(k, j) from lane
// j + 16 k, and returns D(i, j) in lane j + 16 (i % 4), register i / 4; so
// acc[bm][bn][q] is element (row 16 bm + (lane >> 4) + 4 q, col 16 bn + (lane & 15)).
template <bool TRANSB>
__device__ __forceinline__ void gemm64_f64(const double *__restrict__ A, int64_t lda,
                                           const double *__restrict__ B, int64_t ldb, int k0,
                                           int k1, d4 acc[2][2], double *sA, double *sB) {
  // sA, sB: two LDS buffers of KS64 x LDP each; the next k-stage is loaded into
  // registers while the current one is multiplied.
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  double ra[4], rb[4];
  auto fetch = [&](int k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {                      // A: 64 rows x 16 k
      const int m = tid & 63, kk = (tid >> 6) + 4 * q;
      ra[q] = A[(int64_t)(k + kk) * lda + m];
    }
    if (!TRANSB) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {                    // B: contiguous in k
        const int kk = tid & 15, nn = (tid >> 4) + 16 * q;
        rb[q] = B[(int64_t)nn * ldb + k + kk];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {                    // B: contiguous in n
        const int nn = tid & 63, kk = (tid >> 6) + 4 * q;
        rb[q] = B[(int64_t)(k + kk) * ldb + nn];
      }
    }
  };
  auto stage = [&](int b) {
    double *a = sA + b * KS64 * LDP, *bb = sB + b * KS64 * LDP;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = tid & 63, kk = (tid >> 6) + 4 * q;
      a[kk * LDP + m] = ra[q];
    }
    if (!TRANSB) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = tid & 15, nn = (tid >> 4) + 16 * q;
        bb[kk * LDP + nn] = rb[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int nn = tid & 63, kk = (tid >> 6) + 4 * q;
        bb[kk * LDP + nn] = rb[q];
      }
    }
  };
  if (k0 >= k1) return;
  fetch(k0);
  stage(0);
  __syncthreads();
  int b = 0;
  for (int k = k0; k < k1; k += KS64) {
    const bool more = k + KS64 < k1;
    if (more) fetch(k + KS64);
    const double *a = sA + b * KS64 * LDP, *bb = sB + b * KS64 * LDP;
#pragma unroll
    for (int kk = 0; kk < KS64; kk += 4) {
      const int kr = kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = a[kr * LDP + wm + 16 * t + (lane & 15)];
        bv[t] = bb[kr * LDP + wn + 16 * t + (lane & 15)];
      }
#pragma unroll
      for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn)
          acc[bm][bn] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bm], bv[bn], acc[bm][bn], 0, 0, 0);
    }
    if (more) stage(b ^ 1);
    __syncthreads();
    b ^= 1;
  }
}

__device__ __forceinline__ void acc_zero(d4 acc[2][2]) {
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) acc[bm][bn] = d4{0.0, 0.0, 0.0, 0.0};
}

// Visit the 64x64 tile owned by this thread: f(r, c, value).
template <typename F>
__device__ __forceinline__ void acc_foreach(d4 acc[2][2], F f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        f(wm + 16 * bm + (lane >> 4) + 4 * q, wn + 16 * bn + (lane & 15), acc[bm][bn][q]);
}

__device__ __forceinline__ void tri_index(int x, int &ti, int &tj) {   // x -> (ti >= tj)
  int t = (int)((sqrtf(8.0f * (float)x + 1.0f) - 1.0f) * 0.5f);
  while ((t + 1) * (t + 2) / 2 <= x) ++t;
  while (t * (t + 1) / 2 > x) --t;
  ti = t;
  tj = x - t * (t + 1) / 2;
}

// Tile kernels over a (tiles, submatrices) grid take their (tile, submatrix) pair
// through xcd_remap of the flat workgroup id, so that the tiles of one submatrix run
// on one XCD and share its panels in that XCD's L2.
__device__ __forceinline__ void remap_tile_sub(int &tile, int &sub) {
  const int nx = (int)gridDim.x;
  const int l = xcd_remap((int)blockIdx.x + nx * (int)blockIdx.y, nx * (int)gridDim.y);
  tile = l % nx;
  sub = l / nx;
}

#define SUB_PTRS SUB_PTRS_AT(blockIdx.y)
#define SUB_PTRS_AT(k)                                                         \
  const SubDesc d = desc[k];                                                   \
  const int ld = d.npad;                                                       \
  double *Hb = reinterpret_cast<double *>(ws + d.off_h);                       \
  double *Sb = reinterpret_cast<double *>(ws + d.off_s);                       \
  double *Dinv = reinterpret_cast<double *>(ws + d.off_diag);                  \
  double *Tmp = Dinv + (int64_t)ld * NB;                                       \
  (void)Hb; (void)Sb; (void)Dinv; (void)Tmp;

// ------------------------------------------------------------------ Cholesky

// Unblocked Cholesky of the 64 x 64 diagonal block j and the inverse of its factor,
// both right-looking with one barrier per column:
//   factor:  A[r][s] -= A[r][c] A[s][c] / A[c][c]  (r >= s > c); afterwards
//            L[c][c] = sqrt(A[c][c]), L[r][c] = A[r][c] / L[c][c]
//   inverse: Y = I;  Y[r][k] -= A[r][q] Y[q][k] / A[q][q]  (r > q >= k); afterwards
//            L^-1[r][k] = Y[r][k] / L[r][r]
// (L X = I solved row by row: row q of Y is final once the columns before q are done).
// The block lives in registers: thread (tr, tc) = (tid / 16, tid % 16) holds rows
// tr + 16 i and columns tc + 16 jj (i, jj < 4); column c of A (row q of Y) is
// published through a double-buffered LDS vector by the threads that hold it.
__global__ __launch_bounds__(256) void chol_diag_kernel(const SubDesc *__restrict__ desc,
                                                        SubState *__restrict__ st, char *ws,
                                                        int jb) {
  SUB_PTRS
  const int j = jb * NB;
  if (j >= ld) return;
  __shared__ double sA[NB * LDP];       // the factored block (for the inverse)
  __shared__ double vec[2][NB];
  __shared__ double sD[NB];
  __shared__ int bad;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  if (tid == 0) bad = 0;
  double a[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
      a[i][jj] = Sb[(int64_t)(j + tc + 16 * jj) * ld + j + tr + 16 * i];
  // factor: step c = 16 jj + cc; the holders of column c (tc == cc) publish it
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
#pragma unroll 1
    for (int cc = 0; cc < 16; ++cc) {
      const int c = 16 * jj + cc, b = c & 1;
      if (tc == cc) {
#pragma unroll
        for (int i = 0; i < 4; ++i) vec[b][tr + 16 * i] = a[i][jj];
      }
      __syncthreads();
      double dc = vec[b][c];
      if (!(dc > 0.0)) {                  // not positive definite: flag, keep going finite
        if (tid == 0) bad = 1;
        dc = 1.0;
      }
      const double inv = 1.0 / dc;
      double cr[4], cs[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) cr[i] = vec[b][tr + 16 * i] * inv;
#pragma unroll
      for (int q = 0; q < 4; ++q) cs[q] = vec[b][tc + 16 * q];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = tr + 16 * i, s2 = tc + 16 * q;
          if (s2 > c && r >= s2) a[i][q] -= cr[i] * cs[q];
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) sA[(tr + 16 * i) * LDP + tc + 16 * jj] = a[i][jj];
  __syncthreads();
  if (tid < NB) {
    const double dc = sA[tid * LDP + tid];
    sD[tid] = dc > 0.0 ? sqrt(dc) : 1.0;
  }
  double y[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) y[i][jj] = (tr + 16 * i == tc + 16 * jj) ? 1.0 : 0.0;
  // inverse: step q = 16 ii + qq; the holders of row q of Y (tr == qq) publish it
#pragma unroll
  for (int ii = 0; ii < 4; ++ii) {
#pragma unroll 1
    for (int qq = 0; qq < 16; ++qq) {
      const int q = 16 * ii + qq, b = q & 1;
      if (tr == qq) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) vec[b][tc + 16 * jj] = y[ii][jj];
      }
      __syncthreads();
      double dq = sA[q * LDP + q];
      if (!(dq > 0.0)) dq = 1.0;
      const double inv = 1.0 / dq;
      double ar[4], yq[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) ar[i] = sA[(tr + 16 * i) * LDP + q] * inv;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) yq[jj] = vec[b][tc + 16 * jj];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int r = tr + 16 * i, k = tc + 16 * jj;
          if (r > q && k <= q) y[i][jj] -= ar[i] * yq[jj];
        }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int r = tr + 16 * i, c = tc + 16 * jj;
      const double l = r > c ? sA[r * LDP + c] / sD[c] : (r == c ? sD[c] : 0.0);
      Sb[(int64_t)(j + c) * ld + j + r] = l;
      Dinv[(int64_t)jb * NB * NB + r + c * NB] = r >= c ? y[i][jj] / sD[r] : 0.0;
    }
  if (tid == 0 && bad) st[blockIdx.y].status = NOLSM_ENOTSPD;
}

// F32: the rows below the diagonal block also go, rounded to FP32, to the panel copy
// that the FP32 trailing update reads (column (jb - jb0) 64 + c of the outer block
// that starts at column block jb0, leading dimension ld, in the iteration arena,
// which is free during the factorisation).
template <bool F32>
__global__ __launch_bounds__(256) void chol_panel_kernel(const SubDesc *__restrict__ desc,
                                                         char *ws, int jb, int jb0) {
  SUB_PTRS
  const int j = jb * NB;
  const int i0 = j + NB + blockIdx.x * 64;
  if (i0 >= ld) return;
  __shared__ double sm[4 * KS64 * LDP];         // the two stage buffers, then the result
  static_assert(4 * KS64 * LDP >= NB * LDP, "result tile fits the stage buffers");
  d4 acc[2][2];
  acc_zero(acc);
  // out(r, c) = sum_s P(r, s) Linv_jj(c, s);  B(k=s, n=c) = Dinv[c + s*64]
  gemm64_f64<true>(Sb + (int64_t)j * ld + i0, ld, Dinv + (int64_t)jb * NB * NB, NB, 0, NB, acc,
                   sm, sm + 2 * KS64 * LDP);
  // through LDS (column c at sm[c LDP + r]; the product's last barrier has passed), then
  // one column of 64 rows per wave and store: 512 contiguous bytes (256 of the copy)
  acc_foreach(acc, [&](int r, int c, double v) { sm[c * LDP + r] = v; });
  __syncthreads();
  float *P32 = reinterpret_cast<float *>(ws + d.off_lo) + (int64_t)(jb - jb0) * NB * ld;
  const int lane = threadIdx.x & 63;
  for (int c = threadIdx.x >> 6; c < NB; c += 4) {
    const double v = sm[c * LDP + lane];
    Sb[(int64_t)(j + c) * ld + i0 + lane] = v;
    if (F32) P32[(int64_t)c * ld + i0 + lane] = (float)v;
  }
}

// A[r, c] -= sum_{k0 <= s < k1} L[r, s] L[c, s] on the 64 x 64 tiles (ti, tj) with
// tj in [cb0, cb1) and ti >= tj (lower tiles only).  blockIdx.x enumerates the
// rectangle ti in [cb0, nb_max), tj in [cb0, cb1) column by column; tiles above
// the diagonal or beyond this submatrix exit at once.
// (FP64 factorisation; with the FP32 tiles chol_update128_kernel does this step.)
__global__ __launch_bounds__(256) void chol_update_kernel(const SubDesc *__restrict__ desc,
                                                          char *ws, int k0, int k1, int cb0,
                                                          int cb1, int rows) {
  SUB_PTRS
  const int ti = cb0 + (int)blockIdx.x % rows, tj = cb0 + (int)blockIdx.x / rows;
  const int nb = ld / 64;
  if (ti < tj || ti >= nb || tj >= nb || k0 >= ld) return;
  const int r0 = ti * 64, c0 = tj * 64;
  // C(r, c) -= sum_s L(r0 + r, s) L(c0 + c, s);  B(k=s, n=c) = S[s*ld + c0 + c]
  __shared__ double sA[2 * KS64 * LDP], sB[2 * KS64 * LDP];
  d4 acc[2][2];
  acc_zero(acc);
  gemm64_f64<true>(Sb + (int64_t)k0 * ld + r0, ld, Sb + (int64_t)k0 * ld + c0, ld, 0, k1 - k0,
                   acc, sA, sB);
  acc_foreach(acc, [&](int r, int c, double v) {
    double *p = Sb + (int64_t)(c0 + c) * ld + r0 + r;
    *p = *p - v;
  });
}

// 128 x 128 FP64 tile product for the blocked set-up steps:
//   acc(r, c) += sum_{k0 <= k < k1} A[k lda + r] B(k, c),   0 <= r, c < 128,
// B(k, c) = B[k ldb + c], or B[c ldb + k] when TB; rows r >= nA and columns
// c >= nB read as zero (k1 - k0: a multiple of KS64).
// An FP64 MFMA issues at about half rate from a single wave (measured: 35 TF/s with
// one wave per SIMD, 75-78 TF/s with two), so the workgroup has eight waves, two
// per SIMD; wave w owns rows 32 (w >> 1) .. + 31 and columns 64 (w & 1) .. + 63 as
// 2 x 4 blocks of 16 x 16 (layout as in gemm64_f64).  The next k-stage is loaded
// into registers while the current one is multiplied (two LDS buffers).
constexpr int LDQ = 128 + 1;        // padded LDS row (doubles) of the 128-wide stages
constexpr int T128_THREADS = 512;
typedef double Stage128[KS64 * LDQ];

// A wave whose rows all lie at or past nA, whose columns all lie at or past nB, or
// (lower) whose block lies above the diagonal of a diagonal tile issues no MFMAs (its
// accumulators stay zero and the function returns true); it still loads its share of
// every stage, so the MFMA pipe of its SIMD serves the other waves.
template <bool TB>
__device__ __forceinline__ bool tile128_f64(const double *__restrict__ A, int64_t lda,
                                            const double *__restrict__ B, int64_t ldb, int nA,
                                            int nB, int k0, int k1, d4 acc[2][4], Stage128 *sA,
                                            Stage128 *sB, bool lower = false) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 64;
  const bool idle = wm >= nA || wn >= nB || (lower && wm + 31 < wn);
  // element q of this thread's share of a stage: row m = idx & 127, k = idx >> 7
  double ra[4], rb[4];
  auto load = [&](int k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + T128_THREADS * q, m = idx & 127, kk = idx >> 7;
      ra[q] = (m < nA) ? A[(int64_t)(k + kk) * lda + m] : 0.0;
      if (!TB) {
        rb[q] = (m < nB) ? B[(int64_t)(k + kk) * ldb + m] : 0.0;
      } else {                                   // 16 contiguous k of one column
        const int kt = idx & 15, n = idx >> 4;
        rb[q] = (n < nB) ? B[(int64_t)n * ldb + k + kt] : 0.0;
      }
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + T128_THREADS * q, m = idx & 127, kk = idx >> 7;
      sA[b][kk * LDQ + m] = ra[q];
      if (!TB)
        sB[b][kk * LDQ + m] = rb[q];
      else
        sB[b][(idx & 15) * LDQ + (idx >> 4)] = rb[q];
    }
  };
  if (k0 >= k1) return idle;
  load(k0);
  store(0);
  __syncthreads();
  int b = 0;
  for (int k = k0; k < k1; k += KS64) {
    const bool more = k + KS64 < k1;
    if (more) load(k + KS64);
    if (!idle) {
#pragma unroll
      for (int kk = 0; kk < KS64; kk += 4) {
        const int kr = kk + (lane >> 4);
        double a[2], bb[4];
#pragma unroll
        for (int t = 0; t < 2; ++t) a[t] = sA[b][kr * LDQ + wm + 16 * t + (lane & 15)];
#pragma unroll
        for (int t = 0; t < 4; ++t) bb[t] = sB[b][kr * LDQ + wn + 16 * t + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
      }
    }
    if (more) store(b ^ 1);
    __syncthreads();
    b ^= 1;
  }
  return idle;
}

// Visit this thread's elements of a 128 x 128 tile: f(r, c, value).
template <typename F>
__device__ __forceinline__ void acc128_foreach(d4 acc[2][4], F f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 64;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        f(wm + 16 * i + (lane >> 4) + 4 * q, wn + 16 * j + (lane & 15), acc[i][j][q]);
}

// The same 128 x 128 tile product on FP32 MFMAs (v_mfma_f32_16x16x4_f32, twice the
// FP64 rate): the FP64 operands are rounded to FP32 as they are staged in LDS and the
// products are summed in FP32; the caller applies the result to its FP64 matrix.
// Rounding the factor's trailing updates and the inverse's outer products this way
// leaves L^-1 S L^-T - I at a few 1e-7 (an FP32 factorisation), which moves the
// density columns by about 1e-7 and a molecule's energy by about 1e-7 Ha/atom, far
// below the FP16 rounding of the sign iteration.  The input layout of the FP32
// instruction is that of the FP64 one; its output puts D(i, j) in lane j + 16 (i / 4),
// register i % 4.  LDS rows are padded by 16 floats, so the four 16-lane groups of a
// fragment read (consecutive k) fall on different banks.
constexpr int LDQF = 128 + 16;
constexpr int KSF = 16;             // k per LDS stage of the FP32 tiles (32 measured no faster)
typedef float Stage128f[KSF * LDQF];

template <bool TB, typename TA, typename TBT>
__device__ __forceinline__ bool tile128_f32(const TA *__restrict__ A, int64_t lda,
                                            const TBT *__restrict__ B, int64_t ldb, int nA,
                                            int nB, int k0, int k1, f4x acc[2][4], Stage128f *sA,
                                            Stage128f *sB, bool lower = false) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 64;
  const bool idle = wm >= nA || wn >= nB || (lower && wm + 31 < wn);
  constexpr int NQ = KSF * 128 / T128_THREADS;     // elements per thread per operand and stage
  // An FP32 operand (not transposed) is read 4 rows at a time: thread t takes rows
  // 4 (t % 32) .. + 3 of stage row t / 32 (the NQ = 4 elements of one 16-byte load;
  // its leading dimension and base are multiples of 4 floats).
  constexpr bool VA = std::is_same<TA, float>::value;
  constexpr bool VB = std::is_same<TBT, float>::value && !TB;
  static_assert(!(VA || VB) || NQ == 4, "4-wide FP32 staging needs 4 elements per thread");
  TA ra[NQ];
  TBT rb[NQ];
  auto load4 = [&](const float *__restrict__ X, int64_t ldx, int nX, int k, float *r) {
    const int kk = tid >> 5, m4 = (tid & 31) * 4;
    const bool kin = k + kk < k1;
    if (kin && m4 + 3 < nX) {
      const f4x v = *reinterpret_cast<const f4x *>(X + (int64_t)(k + kk) * ldx + m4);
#pragma unroll
      for (int q = 0; q < 4; ++q) r[q] = v[q];
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        r[q] = (kin && m4 + q < nX) ? X[(int64_t)(k + kk) * ldx + m4 + q] : 0.0f;
    }
  };
  auto load = [&](int k) {
    if constexpr (VA) load4(A, lda, nA, k, ra);
    if constexpr (VB) load4(B, ldb, nB, k, rb);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int idx = tid + T128_THREADS * q, m = idx & 127, kk = idx >> 7;
      if constexpr (!VA) ra[q] = (m < nA && k + kk < k1) ? A[(int64_t)(k + kk) * lda + m] : (TA)0;
      if constexpr (VB) {
      } else if constexpr (!TB) {
        rb[q] = (m < nB && k + kk < k1) ? B[(int64_t)(k + kk) * ldb + m] : (TBT)0;
      } else {
        const int kt = idx & (KSF - 1), n = idx / KSF;
        rb[q] = (n < nB && k + kt < k1) ? B[(int64_t)n * ldb + k + kt] : (TBT)0;
      }
    }
  };
  auto store = [&](int b) {
    const int kk4 = tid >> 5, m4 = (tid & 31) * 4;
    if constexpr (VA)
      *reinterpret_cast<f4x *>(&sA[b][kk4 * LDQF + m4]) = f4x{ra[0], ra[1], ra[2], ra[3]};
    if constexpr (VB)
      *reinterpret_cast<f4x *>(&sB[b][kk4 * LDQF + m4]) = f4x{rb[0], rb[1], rb[2], rb[3]};
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int idx = tid + T128_THREADS * q, m = idx & 127, kk = idx >> 7;
      if constexpr (!VA) sA[b][kk * LDQF + m] = (float)ra[q];
      if constexpr (VB) {
      } else if constexpr (!TB) {
        sB[b][kk * LDQF + m] = (float)rb[q];
      } else {
        sB[b][(idx & (KSF - 1)) * LDQF + idx / KSF] = (float)rb[q];
      }
    }
  };
  if (k0 >= k1) return idle;
  load(k0);
  store(0);
  __syncthreads();
  int b = 0;
  for (int k = k0; k < k1; k += KSF) {
    const bool more = k + KSF < k1;
    if (more) load(k + KSF);
    if (!idle) {
#pragma unroll
      for (int kk = 0; kk < KSF; kk += 4) {
        const int kr = kk + (lane >> 4);
        float a[2], bb[4];
#pragma unroll
        for (int t = 0; t < 2; ++t) a[t] = sA[b][kr * LDQF + wm + 16 * t + (lane & 15)];
#pragma unroll
        for (int t = 0; t < 4; ++t) bb[t] = sB[b][kr * LDQF + wn + 16 * t + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bb[j], acc[i][j], 0, 0, 0);
      }
    }
    if (more) store(b ^ 1);
    __syncthreads();
    b ^= 1;
  }
  return idle;
}

// One 128 x 128 tile product on FP64 MFMAs (the FP64 factorisation option; the FP32
// tiles go through tile128_f32_staged); f(r, c, value) visits the result unless every
// wave was idle (then nothing is to be applied).
template <bool TB, typename F>
__device__ __forceinline__ void tile128(const double *__restrict__ A, int64_t lda,
                                        const double *__restrict__ B, int64_t ldb, int nA, int nB,
                                        int k0, int k1, bool lower, F f) {
  __shared__ Stage128 sA[2], sB[2];
  d4 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  if (tile128_f64<TB>(A, lda, B, ldb, nA, nB, k0, k1, acc, sA, sB, lower)) return;
  acc128_foreach(acc, f);
}

// The FP32 tile product with its result handed to g(r, c, value) in coalesced order:
// staged through LDS 64 columns at a time (column c at t[c LT + r]), then each wave
// takes one column of 128 rows in two 64-lane runs, or with ROWMAJOR one row of 64
// columns per run.  Every wave takes part in the barriers; a wave with nothing to
// multiply holds zeros, so g sees every element of the tile's column halves that
// hold live columns (c < nB; it applies its own bounds).
template <bool TB, bool ROWMAJOR, typename TA, typename TBT, typename G>
__device__ __forceinline__ void tile128_f32_staged(const TA *__restrict__ A, int64_t lda,
                                                   const TBT *__restrict__ B, int64_t ldb,
                                                   int nA, int nB, int k0, int k1, bool lower,
                                                   G g) {
  __shared__ __align__(16) float sm[4 * KSF * LDQF];
  Stage128f *sA = reinterpret_cast<Stage128f *>(sm), *sB = sA + 2;
  constexpr int LT = 128 + 4;
  static_assert(4 * KSF * LDQF >= 64 * LT, "half tile fits the stage buffers");
  f4x acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4x{0.0f, 0.0f, 0.0f, 0.0f};
  tile128_f32<TB>(A, lda, B, ldb, nA, nB, k0, k1, acc, sA, sB, lower);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 32;
  for (int h = 0; h < 2; ++h) {
    if (64 * h >= nB) break;           // no live columns in this half (uniform)
    __syncthreads();
    if ((w & 1) == h) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            sm[(16 * j + (lane & 15)) * LT + wm + 16 * i + 4 * (lane >> 4) + q] = acc[i][j][q];
    }
    __syncthreads();
    if (!ROWMAJOR) {
      for (int c = w; c < 64; c += T128_THREADS / 64)
#pragma unroll
        for (int rr = lane; rr < 128; rr += 64) g(rr, 64 * h + c, (double)sm[c * LT + rr]);
    } else {
      for (int r = w; r < 128; r += T128_THREADS / 64)
        g(r, 64 * h + lane, (double)sm[lane * LT + r]);
    }
  }
}

// Trailing update of the outer Cholesky blocks on 128 x 128 tiles:
//   A[r, c] -= sum_{k0 <= s < k1} L[r, s] L[c, s],  tiles (ti, tj) of 128 with ti >= tj
// starting at row/column m0 (a multiple of 128).  A 64 x 64 FP64 tile reads
// 6.5 flop per byte of its panels; the 128 x 128 tile doubles that.
template <bool F32>
__global__ __launch_bounds__(T128_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
void chol_trail_kernel(const SubDesc *__restrict__ desc, char *ws, int k0, int k1, int m0,
                       int rows) {
  int tile, sub;
  remap_tile_sub(tile, sub);
  SUB_PTRS_AT(sub)
  const int ti = tile % rows, tj = tile / rows;
  if (ti < tj || k0 >= ld) return;
  const int r0 = m0 + ti * 128, c0 = m0 + tj * 128;
  if (r0 >= ld || c0 >= ld) return;
  auto apply = [&](int r, int c, double v) {
    if (r0 + r < ld && c0 + c < ld) {
      double *p = Sb + (int64_t)(c0 + c) * ld + r0 + r;
      *p = *p - v;
    }
  };
  if constexpr (F32) {      // the outer block's columns from their FP32 copy (chol_panel)
    // (in a diagonal tile the part above the diagonal is left alone: nothing reads it)
    const float *P32 = reinterpret_cast<const float *>(ws + d.off_lo);
    tile128_f32_staged<false, false>(P32 + r0, ld, P32 + c0, ld, ld - r0, ld - c0, 0, k1 - k0,
                                     ti == tj, [&](int r, int c, double v) {
                                       if (ti != tj || r >= c) apply(r, c, v);
                                     });
  } else {
    tile128<false>(Sb + r0, ld, Sb + c0, ld, ld - r0, ld - c0, k0, k1, ti == tj, apply);
  }
}

// Left-looking update of column block cb inside an outer block on the FP32 tiles:
//   A[r, c] -= sum_{k0 <= s < k1} L[r, s] L[c, s],  r >= 64 cb, c in column block cb,
// in 128-row tiles (rows 64 cb + 128 x .. + 127) of the 8-wave FP32 tile product with
// 64 live columns (the waves of the other 64 only share the loads), operands from
// the outer block's FP32 panel copy (chol_panel: column s - k0, rows below the
// diagonal block of s, which covers every row read here), results through LDS.
__global__ __launch_bounds__(T128_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
void chol_update128_kernel(const SubDesc *__restrict__ desc, char *ws, int k0, int k1, int cb) {
  int tile, sub;
  remap_tile_sub(tile, sub);
  SUB_PTRS_AT(sub)
  const int c0 = cb * NB, r0 = c0 + tile * 128;
  if (r0 >= ld || k0 >= ld) return;
  const float *P32 = reinterpret_cast<const float *>(ws + d.off_lo);
  tile128_f32_staged<false, false>(P32 + r0, ld, P32 + c0, ld, ld - r0, NB, 0, k1 - k0, false,
                                   [&](int r, int c, double v) {
                                     if (c < NB && r0 + r < ld) {
                                       double *p = Sb + (int64_t)(c0 + c) * ld + r0 + r;
                                       *p = *p - v;
                                     }
                                   });
}

// ------------------------------------------------------------------ L^-1 in place

__global__ __launch_bounds__(256) void trtri_diag_kernel(const SubDesc *__restrict__ desc,
                                                         char *ws) {
  SUB_PTRS
  const int jb = blockIdx.x;
  const int j = jb * NB;
  if (j >= ld) return;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e & 63, c = e >> 6;
    Sb[(int64_t)(j + c) * ld + j + r] = Dinv[(int64_t)jb * NB * NB + r + c * NB];
  }
}

// Tmp[i, c] = sum_s L[i, j + s] Linv_jj[s, c]  for rows j + 64 <= i < iend
__global__ __launch_bounds__(256) void trtri_panel_kernel(const SubDesc *__restrict__ desc,
                                                          char *ws, int jb, int iend) {
  SUB_PTRS
  const int j = jb * NB;
  const int i0 = j + NB + blockIdx.x * 64;
  if (i0 >= ld || i0 >= iend) return;
  __shared__ double sA[2 * KS64 * LDP], sB[2 * KS64 * LDP];
  d4 acc[2][2];
  acc_zero(acc);
  gemm64_f64<false>(Sb + (int64_t)j * ld + i0, ld, Dinv + (int64_t)jb * NB * NB, NB, 0, NB, acc,
                    sA, sB);
  acc_foreach(acc, [&](int r, int c, double v) { Tmp[(int64_t)c * ld + i0 + r] = v; });
}

// Linv[i, j-block] = - sum_{k = j+64}^{i-block end} Linv[i, k] Tmp[k, :],  j + 64 <= i < iend
__global__ __launch_bounds__(256) void trtri_update_kernel(const SubDesc *__restrict__ desc,
                                                           char *ws, int jb, int iend) {
  SUB_PTRS
  const int j = jb * NB;
  const int i0 = j + NB + blockIdx.x * 64;
  if (i0 >= ld || i0 >= iend) return;
  __shared__ double sA[2 * KS64 * LDP], sB[2 * KS64 * LDP];
  d4 acc[2][2];
  acc_zero(acc);
  gemm64_f64<false>(Sb + i0, ld, Tmp, ld, j + NB, i0 + 64, acc, sA, sB);
  acc_foreach(acc, [&](int r, int c, double v) { Sb[(int64_t)(j + c) * ld + i0 + r] = -v; });
}

// Outer step of the two-level inverse.  Once the diagonal block X_JJ = L_JJ^-1 of
// the outer block J = [J0, J0 + TW) is in place and the columns right of it hold
// L^-1, the rows i >= J1 = J0 + TW of block column J follow from X L = I:
//   X[i, J] = - sum_{J1 <= k <= i} X[i, k] T[k, :],   T = L[J1:, J] X_JJ.
// T (rows k >= J1, TW columns, row major) lives in the iteration arena, which is
// free until the set-up products.  Both products run on 128 x 128 tiles
// (blockIdx.x = row tile + rows * column tile, two column tiles).
constexpr int TW = 256;                 // outer block width of the inverse

template <bool F32>
__global__ __launch_bounds__(T128_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
void trtri_outer_t_kernel(const SubDesc *__restrict__ desc, char *ws, int J0, int rows) {
  int tile, sub;
  remap_tile_sub(tile, sub);
  SUB_PTRS_AT(sub)
  const int J1 = J0 + TW;
  const int ti = tile % rows, tj = tile / rows;
  const int r0 = J1 + ti * 128, c0 = tj * 128;
  if (r0 >= ld) return;
  // T[r0 + r, c0 + c] = sum_s L[r0 + r, J0 + s] X_JJ[s, c0 + c];  X_JJ[s, c] = 0 for s < c
  // (an all-idle tile has no rows below ld: nothing to store); FP32 with the FP32 tiles,
  // which is how trtri_outer_x reads it then
  typedef typename std::conditional<F32, float, double>::type TT;
  TT *T = reinterpret_cast<TT *>(ws + d.off_lo);
  auto put = [&](int r, int c, double v) {
    if (r0 + r < ld) T[(int64_t)(r0 + r - J1) * TW + c0 + c] = (TT)v;
  };
  if constexpr (F32)        // T is row major: stored a row at a time
    tile128_f32_staged<true, true>(Sb + (int64_t)J0 * ld + r0, ld,
                                   Sb + (int64_t)(J0 + c0) * ld + J0, ld, ld - r0, 128, c0, TW,
                                   false, put);
  else
    tile128<true>(Sb + (int64_t)J0 * ld + r0, ld, Sb + (int64_t)(J0 + c0) * ld + J0, ld,
                  ld - r0, 128, c0, TW, false, put);
}

template <bool F32>
__global__ __launch_bounds__(T128_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
void trtri_outer_x_kernel(const SubDesc *__restrict__ desc, char *ws, int J0, int rows) {
  int tile, sub;
  remap_tile_sub(tile, sub);
  SUB_PTRS_AT(sub)
  const int J1 = J0 + TW;
  const int ti = tile % rows, tj = tile / rows;
  const int r0 = J1 + ti * 128, c0 = tj * 128;
  if (r0 >= ld) return;
  typedef typename std::conditional<F32, float, double>::type TT;
  const TT *T = reinterpret_cast<const TT *>(ws + d.off_lo);
  const int kend = (r0 + 128 < ld ? r0 + 128 : ld) - J1;       // X[i, k] = 0 for k > i
  auto put = [&](int r, int c, double v) {
    if (r0 + r < ld) Sb[(int64_t)(J0 + c0 + c) * ld + r0 + r] = -v;
  };
  if constexpr (F32)
    tile128_f32_staged<false, false>(Sb + (int64_t)J1 * ld + r0, ld, T + c0, TW, ld - r0, 128,
                                     0, kend, false, put);
  else
    tile128<false>(Sb + (int64_t)J1 * ld + r0, ld, T + c0, TW, ld - r0, 128, 0, kend, false,
                   put);
}

__global__ __launch_bounds__(256) void zero_upper_kernel(const SubDesc *__restrict__ desc,
                                                         char *ws) {
  SUB_PTRS
  const int c = blockIdx.x;
  if (c >= ld) return;
  for (int r = threadIdx.x; r < c; r += 256) Sb[(int64_t)c * ld + r] = 0.0;
}

// ------------------------------------------------------------------ M = L^-1 H L^-T

// FP32 operands of the set-up products in the iteration arena: buffer 0 = L^-T
// (the transpose of L^-1, through an LDS tile), buffer 1 = H.
__global__ __launch_bounds__(256) void prep_products_kernel(const SubDesc *__restrict__ desc,
                                                            char *ws) {
  SUB_PTRS
  const int nt = ld / 64;
  if ((int)blockIdx.x >= nt * nt) return;
  const int bi = blockIdx.x / nt, bj = blockIdx.x % nt;
  float *Lt = reinterpret_cast<float *>(ws + d.off_lo);
  float *H32 = Lt + (int64_t)ld * ld;
  __shared__ float tile[64][65];
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e & 63, c = e >> 6;
    const int64_t o = (int64_t)(bj * 64 + c) * ld + bi * 64 + r;
    tile[c][r] = (float)Sb[o];
    H32[o] = (float)Hb[o];
  }
  __syncthreads();
  // L^-T(bj*64 + c, bi*64 + r) = L^-1(bi*64 + r, bj*64 + c)
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int c = e & 63, r = e >> 6;
    Lt[(int64_t)(bi * 64 + r) * ld + bj * 64 + c] = tile[c][r];
  }
}


// Split FP16 operand of the set-up products for L^-1: buffer 0, row r = L^-1(r, :)
// (through an LDS tile, since L^-1 is stored by columns), hi parts then lo parts,
// k-blocked (split_index).  (Buffer 1, the rows of H, is written by the gather.)  Every thread
// converts four consecutive elements: 8-byte stores of hi and of lo.  Blocks above
// the diagonal block are zero in L^-1 (its upper triangle is cleared before the
// inverse), so they are written without being read.
typedef _Float16 h4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void prep_split_kernel(const SubDesc *__restrict__ desc,
                                                         char *ws) {
  SUB_PTRS
  const int nt = ld / 64;
  if ((int)blockIdx.x >= nt * nt) return;
  const int bi = blockIdx.x / nt, bj = blockIdx.x % nt;
  _Float16 *Ls = reinterpret_cast<_Float16 *>(ws + d.off_lo);
  const int64_t llo = (int64_t)ld * ld;                    // lo part after the hi part
  if (bi < bj) {
    const h4 z = {(_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f};
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      _Float16 *lrow = Ls + split_index(bi * 64 + (e >> 4), bj * 64 + (e & 15) * 4, ld);
      *reinterpret_cast<h4 *>(lrow) = z;
      *reinterpret_cast<h4 *>(lrow + llo) = z;
    }
    return;
  }
  __shared__ double tile[64][65];
  for (int e = threadIdx.x; e < 64 * 16; e += 256) {
    const int r4 = (e & 15) * 4, c = e >> 4;
    const int64_t o = (int64_t)(bj * 64 + c) * ld + bi * 64 + r4;   // (bi 64 + r4, bj 64 + c)
    const d4 sv = *reinterpret_cast<const d4 *>(Sb + o);
#pragma unroll
    for (int q = 0; q < 4; ++q) tile[c][r4 + q] = sv[q];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 16; e += 256) {
    const int c4 = (e & 15) * 4, r = e >> 4;
    h4 lh, ll;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      _Float16 a, b;
      split_f16(tile[c4 + q][r], a, b);           // L^-1(bi 64 + r, bj 64 + c4 + q)
      lh[q] = a;
      ll[q] = b;
    }
    _Float16 *lrow = Ls + split_index(bi * 64 + r, bj * 64 + c4, ld);
    *reinterpret_cast<h4 *>(lrow) = lh;
    *reinterpret_cast<h4 *>(lrow + llo) = ll;
  }
}

// keep_spd = 0: clear every status (a new set-up); 1: clear only NOLSM_ENOCONV
__global__ void reset_status_kernel(SubState *__restrict__ st, int K, int keep_spd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  if (!keep_spd || st[i].status == NOLSM_ENOCONV) st[i].status = 0;
}

void launch_reset_status(SubState *st, int K, int keep_spd, hipStream_t s) {
  reset_status_kernel<<<(K + 255) / 256, 256, 0, s>>>(st, K, keep_spd);
}

// ------------------------------------------------------------------ host launcher

template <bool F32>
static void launch_factor(const SubDesc *desc, SubState *st, int K, int max_npad, char *ws,
                          hipStream_t s) {
  const int nbmax = max_npad / NB;
  launch_reset_status(st, K, 0, s);
  // Blocked Cholesky with two levels: inside an outer block of OB columns each
  // 64-wide column block first receives the earlier panels of the same outer block
  // in one update (k = 64, 128, ..., 448: left-looking inside the block), then is
  // factored; the trailing matrix receives the outer block's OB columns in one
  // update (k = OB, right-looking between blocks), which reads and writes it OB / 64
  // times less often than 64-wide steps would.  OB = 512 measured 1.7% faster set-up
  // than 256 on 1,700-1,900-row submatrices (more left-looking work, one FP64
  // read-modify-write of the trailing matrix per 512 columns instead of per 256).
  // The FP32 panel copy of an outer block (OB x npad floats) fits the first
  // iteration buffer (npad^2 floats) since OB <= npad or the block is cut at npad.
  constexpr int OBB = 8;                        // outer block = 8 x 64 columns
  for (int J = 0; J < nbmax; J += OBB) {
    const int Jend = J + OBB < nbmax ? J + OBB : nbmax;
    for (int jb = J; jb < Jend; ++jb) {
      if (jb > J) {
        const int rows = nbmax - jb;
        if (F32)
          chol_update128_kernel<<<dim3((rows * NB + 127) / 128, K), T128_THREADS, 0, s>>>(
              desc, ws, J * NB, jb * NB, jb);
        else
          chol_update_kernel<<<dim3(rows, K), 256, 0, s>>>(desc, ws, J * NB, jb * NB, jb, jb + 1,
                                                           rows);
      }
      chol_diag_kernel<<<dim3(1, K), 256, 0, s>>>(desc, st, ws, jb);
      const int rem = nbmax - jb - 1;
      if (rem > 0) chol_panel_kernel<F32><<<dim3(rem, K), 256, 0, s>>>(desc, ws, jb, J);
    }
    if (Jend < nbmax) {
      // Jend * 64 is a multiple of 512 here, so the 128-wide tiles start aligned
      const int m0 = Jend * NB, rows = (max_npad - m0 + 127) / 128;
      chol_trail_kernel<F32><<<dim3(rows * rows, K), T128_THREADS, 0, s>>>(desc, ws, J * NB,
                                                                        Jend * NB, m0, rows);
    }
  }
  // L^-1 in place, outer blocks of TW columns right to left: the 64-wide steps
  // invert the outer diagonal block, then two 128 x 128-tile products give the
  // block column below it (each outer step reads the finished part of L^-1 once,
  // instead of once per 64-wide column block).
  // the upper triangle still holds S: clear it first, so that the outer steps can
  // read the diagonal block X_JJ as a full (lower-triangular) square
  zero_upper_kernel<<<dim3(max_npad, K), 256, 0, s>>>(desc, ws);
  trtri_diag_kernel<<<dim3(nbmax, K), 256, 0, s>>>(desc, ws);
  for (int J0 = (max_npad - 1) / TW * TW; J0 >= 0; J0 -= TW) {
    const int J1 = J0 + TW, iend = J1 < max_npad ? J1 : max_npad;
    for (int jb = iend / NB - 1; jb >= J0 / NB; --jb) {
      const int rem = iend / NB - jb - 1;
      if (rem <= 0) continue;
      trtri_panel_kernel<<<dim3(rem, K), 256, 0, s>>>(desc, ws, jb, J1);
      trtri_update_kernel<<<dim3(rem, K), 256, 0, s>>>(desc, ws, jb, J1);
    }
    if (J1 < max_npad) {
      const int rows = (max_npad - J1 + 127) / 128;
      trtri_outer_t_kernel<F32><<<dim3(2 * rows, K), T128_THREADS, 0, s>>>(desc, ws, J0, rows);
      trtri_outer_x_kernel<F32><<<dim3(2 * rows, K), T128_THREADS, 0, s>>>(desc, ws, J0, rows);
    }
  }
}

// factor_fp32: the 128 x 128 tile products of the factorisation and the inverse on
// FP32 MFMAs (tile128_f32); otherwise FP64 throughout.
void launch_lit_setup(const SubDesc *desc, const SubState *st, int K, int max_npad, char *ws,
                      hipStream_t s);

// literal: A0 = S^-1 H in place of M (literal.hip; H is gathered in FP64)
void launch_setup(const SubDesc *desc, SubState *st, int K, int max_npad, const TileSet &ts,
                  bool fp32_products, bool factor_fp32, bool literal, char *ws, hipStream_t s) {
  const int nbmax = max_npad / NB;
  if (factor_fp32) launch_factor<true>(desc, st, K, max_npad, ws, s);
  else launch_factor<false>(desc, st, K, max_npad, ws, s);
  if (literal) {
    launch_lit_setup(desc, st, K, max_npad, ws, s);
    return;
  }
  // M = L^-1 H L^-T as two products: U = H L^-T, then M = L^-1 U
  if (!fp32_products) {
    prep_split_kernel<<<dim3(nbmax * nbmax, K), 256, 0, s>>>(desc, ws);
    if (ts.n[4] > 0)
      split_gemm_kernel<SPLIT_FULL><<<ts.n[4], 256, 0, s>>>(ts.t[4], desc, st, ws);
    if (ts.n[5] > 0)
      split_gemm_kernel<SPLIT_SYM><<<ts.n[5], 256, 0, s>>>(ts.t[5], desc, st, ws);
    return;
  }
  prep_products_kernel<<<dim3(nbmax * nbmax, K), 256, 0, s>>>(desc, ws);
  if (ts.n[3] > 0)
    setup_gemm_kernel<EPI_PLAIN_FULL><<<ts.n[3], 256, 0, s>>>(ts.t[3], desc, st, ws);
  if (ts.n[0] > 0)
    setup_gemm_kernel<EPI_PLAIN_SYM><<<ts.n[0], 256, 0, s>>>(ts.t[0], desc, st, ws);
  if (ts.n[2] > 0)
    setup_gemm_kernel<EPI_PLAIN_SYM><<<ts.n[2], 256, 0, s>>>(ts.t[2], desc, st, ws);
}

}  // namespace nolsm
