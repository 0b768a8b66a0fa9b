// The literal form of Eq. 8: the sign iteration on A_k = T_k(S)^-1 T_k(H0) - mu I
// itself, and T_k(D) = 1/2 (I - sign(A_k)) T_k(S)^-1.
//
// The symmetric form (setup.hip, sign.hip) iterates on the congruent matrix
// M_k - mu I = L^-1 (H - mu S) L^-T instead; both give the same T_k(D) in exact
// arithmetic, since every Newton-Schulz iterate is a polynomial in the matrix and
// A_k = L^-T (M_k - mu I) L^T.  The literal form is kept for checking that identity
// on the GPU; the symmetric form is the one that runs fast (its products are
// symmetric, so half of every product is formed, and its iterates stay symmetric).
//
// Set-up (after the factorisation of setup.hip, FP64):
//   P  = L^-1 H          (lit_setup_kernel<false>, FP64, in the iteration arena)
//   A0 = L^-T P = S^-1 H (lit_setup_kernel<true>, FP64 sums, stored in FP32 where the
//                         symmetric form keeps M_k)
// The scale b_k >= rho(A0 - mu I) is the largest column sum of |A0 - mu I| (a
// Gershgorin bound, valid for any matrix), X_0 = (A0 - mu I) / b_k.
// Iteration: A non-symmetric iterate X is kept in buffer 0 with its transpose in
// buffer 1, so that the GEMM kernels, which read both factors as column panels
// (C = A^T B), form X X and X Z from (X^T, X) and (X^T, Z):
//   FULL_SQUARE  Z = c1 I + c3 X X   (buffer 2; residual ||X X - I||_F over every element)
//   PLAIN_FULL   X' = X Z            (buffer 0)
//   transpose    X'^T                (buffer 1)
// every tile of every submatrix (128 x 128 tiles).  At the end the state points at
// buffer 1 (X^T), whose columns are the rows of X, as the panel kernels expect.
// Density columns: V = S^-1[:, own] = L^-T L^-1[:, own] (FP64 sums, FP32 panel),
// W = f(X) V with the panel kernels, T_k(D)[:, own] = 1/2 (V - W) (FP64).
#include "common.h"
#include "ns_gemm.h"

namespace nolsm {

// ------------------------------------------------------------------ set-up

// Out[i0 + i, j0 + j] = sum_k opA(i, k) B[k, j0 + j] on 64 x 64 tiles, FP64;
// TA = false: opA = L^-1 (A(i, k) = Li[k ld + i], zero for k > i), B = H, Out = P;
// TA = true:  opA = L^-T (A(i, k) = Li[i ld + k], zero for k < i), B = P, Out = A0 (FP32).
constexpr int LT = 64, LK = 16;

template <bool TA>
__global__ __launch_bounds__(256) void lit_setup_kernel(const SubDesc *__restrict__ desc,
                                                        const SubState *__restrict__ st,
                                                        char *ws) {
  const SubDesc d = desc[blockIdx.y];
  if (st[blockIdx.y].status != 0) return;
  const int ld = d.npad, nt = ld / LT;
  if ((int)blockIdx.x >= nt * nt) return;
  const int i0 = (blockIdx.x % nt) * LT, j0 = (blockIdx.x / nt) * LT;
  const double *Li = reinterpret_cast<const double *>(ws + d.off_s);
  double *P = reinterpret_cast<double *>(ws + d.off_lo);
  const double *B = TA ? P : reinterpret_cast<const double *>(ws + d.off_h);
  __shared__ double sA[LK][LT + 1], sB[LK][LT + 1];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  const int kb = TA ? i0 : 0, ke = TA ? ld : (i0 + LT < ld ? i0 + LT : ld);
  for (int k0 = kb; k0 < ke; k0 += LK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      if (!TA) {
        const int kk = e / LT, i = e % LT;
        sA[kk][i] = Li[(int64_t)(k0 + kk) * ld + i0 + i];
      } else {
        const int i = e / LK, kk = e % LK;
        sA[kk][i] = Li[(int64_t)(i0 + i) * ld + k0 + kk];
      }
      const int j = e / LK, kk = e % LK;
      sB[kk][j] = B[(int64_t)(j0 + j) * ld + k0 + kk];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < LK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = sA[kk][4 * ty + q];
        b[q] = sB[kk][4 * tx + q];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int64_t o = (int64_t)(j0 + 4 * tx + y) * ld + i0 + 4 * ty + x;
      if (TA) reinterpret_cast<float *>(ws + d.off_h)[o] = (float)acc[x][y];
      else P[o] = acc[x][y];
    }
}

void launch_lit_setup(const SubDesc *desc, const SubState *st, int K, int max_npad, char *ws,
                      hipStream_t s) {
  const int nt = max_npad / LT;
  lit_setup_kernel<false><<<dim3(nt * nt, K), 256, 0, s>>>(desc, st, ws);
  lit_setup_kernel<true><<<dim3(nt * nt, K), 256, 0, s>>>(desc, st, ws);
}

// ------------------------------------------------------------------ iteration

// Buffer 1 <- transpose of buffer 0, in the submatrix's precision, 64 x 64 tiles
// through LDS.  mode 0: every healthy submatrix; 1: the active ones of precision
// prec; 2: the restarting ones (fell_back), if any restart (*cnt).
template <typename TI>
__device__ void lit_transpose_tile(const TI *X, TI *Xt, int ld, int i0, int j0,
                                   float (*t)[LT + 1]) {
  for (int e = threadIdx.x; e < LT * LT; e += 256) {
    const int r = e % LT, c = e / LT;
    t[c][r] = to_f32<TI>(X[(int64_t)(j0 + c) * ld + i0 + r]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < LT * LT; e += 256) {
    const int c = e % LT, r = e / LT;          // Xt(j0 + c, i0 + r) = X(i0 + r, j0 + c)
    Xt[(int64_t)(i0 + r) * ld + j0 + c] = from_f32<TI>(t[c][r]);
  }
}

__global__ __launch_bounds__(256) void lit_transpose_kernel(const SubDesc *__restrict__ desc,
                                                            const SubState *__restrict__ st,
                                                            char *ws, int mode, int prec,
                                                            const unsigned *__restrict__ cnt) {
  const SubDesc d = desc[blockIdx.y];
  const SubState &s = st[blockIdx.y];
  if (s.status != 0) return;
  if (mode == 1 && (!s.active || s.prec != prec)) return;
  if (mode == 2 && (*cnt == 0u || !s.fell_back)) return;
  const int ld = d.npad, nt = ld / LT;
  if ((int)blockIdx.x >= nt * nt) return;
  const int i0 = (blockIdx.x % nt) * LT, j0 = (blockIdx.x / nt) * LT;
  __shared__ float t[LT][LT + 1];
  if (s.prec == P_FP32)
    lit_transpose_tile<float>(buf_ptr<float>(ws, d, 0), buf_ptr<float>(ws, d, 1), ld, i0, j0, t);
  else if (s.prec == P_FP16)
    lit_transpose_tile<_Float16>(buf_ptr<_Float16>(ws, d, 0), buf_ptr<_Float16>(ws, d, 1), ld,
                                 i0, j0, t);
  else
    lit_transpose_tile<__bf16>(buf_ptr<__bf16>(ws, d, 0), buf_ptr<__bf16>(ws, d, 1), ld, i0, j0,
                               t);
}

void launch_lit_transpose(const SubDesc *desc, const SubState *st, int K, int max_npad, char *ws,
                          int mode, int prec, const unsigned *cnt, hipStream_t s) {
  const int nt = max_npad / LT;
  lit_transpose_kernel<<<dim3(nt * nt, K), 256, 0, s>>>(desc, st, ws, mode, prec, cnt);
}

// FULL_SQUARE: Z = c1 I + c3 X X from (X^T, X) into buffer 2; PLAIN_FULL: X' = X Z
// from (X^T, Z) into buffer 0.  Every 128 x 128 tile of every submatrix (tile list 3).
template <typename TI, int EPI>
__global__ __launch_bounds__(256) void lit_gemm_kernel(const Tile *__restrict__ tiles,
                                                       const SubDesc *__restrict__ desc,
                                                       SubState *__restrict__ st, char *ws,
                                                       int prec,
                                                       unsigned long long *__restrict__ flop_units) {
  constexpr int TILE = 128;
  const Tile t = tiles[xcd_remap(blockIdx.x, gridDim.x)];
  SubState &S = st[t.sub];
  if (!S.active || S.prec != prec) return;
  const SubDesc d = desc[t.sub];
  const int ld = d.npad;
  const TI *A = buf_ptr<TI>(ws, d, 1);
  const TI *B = buf_ptr<TI>(ws, d, EPI == EPI_FULL_SQUARE ? 0 : 2);
  TI *Out = buf_ptr<TI>(ws, d, EPI == EPI_FULL_SQUARE ? 2 : 0);
  const int i0 = t.ti * TILE, j0 = t.tj * TILE;
  if (threadIdx.x == 0) {
    const int rows = (ld - i0 < TILE ? ld - i0 : TILE), cols = (ld - j0 < TILE ? ld - j0 : TILE);
    atomicAdd(flop_units, (unsigned long long)((rows / 16) * (cols / 16) * (ld / 64)));
  }
  __shared__ uint4 s0[slot_u4<2>()], s1[slot_u4<2>()], s2[slot_u4<2>()], s3[slot_u4<2>()];
  __shared__ float red[4];
  if (i0 + TILE <= ld && j0 + TILE <= ld)
    ns_gemm_body<TI, EPI, 2, false, 2>(A, B, Out, ld, ld, d.n, i0, j0, S.c1, S.c3, s0, s1, s2, s3,
                                       red, &S.racc);
  else
    ns_gemm_body<TI, EPI, 2, true, 2>(A, B, Out, ld, ld, d.n, i0, j0, S.c1, S.c3, s0, s1, s2, s3,
                                      red, &S.racc);
}

template <int EPI>
static void lit_gemm_t(const Tile *tiles, int ntiles, const SubDesc *desc, SubState *st, char *ws,
                       int prec, unsigned long long *flop_units, hipStream_t s) {
  if (prec == P_FP32)
    lit_gemm_kernel<float, EPI><<<ntiles, 256, 0, s>>>(tiles, desc, st, ws, prec, flop_units);
  else if (prec == P_FP16)
    lit_gemm_kernel<_Float16, EPI><<<ntiles, 256, 0, s>>>(tiles, desc, st, ws, prec, flop_units);
  else
    lit_gemm_kernel<__bf16, EPI><<<ntiles, 256, 0, s>>>(tiles, desc, st, ws, prec, flop_units);
}

void launch_lit_gemm(int square, const Tile *tiles, int ntiles, const SubDesc *desc, SubState *st,
                     char *ws, int prec, unsigned long long *flop_units, hipStream_t s) {
  if (ntiles <= 0) return;
  if (square) lit_gemm_t<EPI_FULL_SQUARE>(tiles, ntiles, desc, st, ws, prec, flop_units, s);
  else lit_gemm_t<EPI_PLAIN_FULL>(tiles, ntiles, desc, st, ws, prec, flop_units, s);
}

__global__ void lit_point_at_transpose_kernel(SubState *__restrict__ st, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) st[i].cur = 1;
}

void launch_lit_finish(SubState *st, int K, hipStream_t s) {
  lit_point_at_transpose_kernel<<<(K + 255) / 256, 256, 0, s>>>(st, K);
}

// ------------------------------------------------------------------ density columns

// V[:, c] = S^-1[:, own_lo + c] = sum_{k >= r} L^-1[k, r] L^-1[k, own_lo + c], FP64 sums,
// stored as the FP32 panel qv; one wave per (row, column), lanes over k.
__global__ __launch_bounds__(256) void lit_panel_v_kernel(const SubDesc *__restrict__ desc,
                                                          const SubState *__restrict__ st,
                                                          char *ws, int qv) {
  const SubDesc d = desc[blockIdx.y];
  if (st[blockIdx.y].status != 0) return;
  const double *Li = reinterpret_cast<const double *>(ws + d.off_s);
  float *V = reinterpret_cast<float *>(ws + d.off_panel) + (int64_t)qv * d.npad * d.m;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int total = d.npad * d.m;
  for (int e = blockIdx.x * 4 + wv; e < total; e += gridDim.x * 4) {
    const int c = e / d.npad, r = e - c * d.npad;
    const double *lr = Li + (int64_t)r * d.npad, *lc = Li + (int64_t)(d.own_lo + c) * d.npad;
    double acc = 0.0;
    for (int k = r + lane; k < d.npad; k += 64) acc += lr[k] * lc[k];
    acc = wave_sum(acc);
    if (lane == 0) V[e] = (float)acc;
  }
}

// Dcol = 1/2 (V - W) in FP64.
__global__ __launch_bounds__(256) void lit_dcol_kernel(const SubDesc *__restrict__ desc,
                                                       const SubState *__restrict__ st, char *ws,
                                                       int qv, int qw) {
  const SubDesc d = desc[blockIdx.y];
  if (st[blockIdx.y].status != 0) return;
  const float *V = reinterpret_cast<const float *>(ws + d.off_panel) + (int64_t)qv * d.npad * d.m;
  const float *W = reinterpret_cast<const float *>(ws + d.off_panel) + (int64_t)qw * d.npad * d.m;
  double *Dc = reinterpret_cast<double *>(ws + d.off_dcol);
  const int total = d.npad * d.m;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256)
    Dc[e] = 0.5 * ((double)V[e] - (double)W[e]);
}

void launch_lit_panel_v(const SubDesc *desc, const SubState *st, int K, char *ws, int qv,
                        hipStream_t s) {
  lit_panel_v_kernel<<<dim3(256, K), 256, 0, s>>>(desc, st, ws, qv);
}

void launch_lit_dcol(const SubDesc *desc, const SubState *st, int K, char *ws, int qv, int qw,
                     hipStream_t s) {
  lit_dcol_kernel<<<dim3(64, K), 256, 0, s>>>(desc, st, ws, qv, qw);
}

}  // namespace nolsm
