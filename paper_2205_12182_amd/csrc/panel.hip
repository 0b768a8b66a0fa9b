// Density columns, write-back and traces.
//
// Only molecule k's own m columns of T_k(D) are written back (paper, Sec. II,
// submatrix method step 3), and in the symmetric form
//   T_k(D)[:, own] = 1/2 L^-T (I - X) L^-1[:, own] = 1/2 L^-T (V - X V),  V = L^-1[:, own],
// so the final refinement of X only has to act on the n x m panel V: s
// Newton-Schulz steps f(X) = 1/2 X (3I - X^2) applied to V cost 3^s panel
// products X P (n^2 m each) instead of full n^3 GEMMs.
//
//   panel_v_kernel     V = L^-1[:, own]                    (FP64 -> FP32)
//   panel_mul_kernel   O = alpha X P + beta Q              (X in its iteration precision, FP32 math)
//   dcol_kernel        Dcol = 1/2 L^-T (V - W)             (FP64)
//   scatter_kernel     block column k of D <- Dcol; per-column Tr contributions (FP64)
//   coltrace / final   Tr(D H), Tr(D S) over the whole pattern, fixed reduction order
#include <mutex>

#include "common.h"

namespace nolsm {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float *panel_ptr(char *ws, const SubDesc &d, int q) {
  return reinterpret_cast<float *>(ws + d.off_panel) + (int64_t)q * d.npad * d.m;
}

__global__ __launch_bounds__(256) void panel_v_kernel(const SubDesc *__restrict__ desc,
                                                      const SubState *__restrict__ st, char *ws,
                                                      int qv) {
  const SubDesc d = desc[blockIdx.y];
  if (st[blockIdx.y].status != 0) return;
  const double *Li = reinterpret_cast<const double *>(ws + d.off_s);
  float *V = panel_ptr(ws, d, qv);
  const int total = d.npad * d.m;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
    const int c = e / d.npad, r = e - c * d.npad;
    V[e] = (float)Li[(int64_t)(d.own_lo + c) * d.npad + r];
  }
}

// O[:, c] = alpha * X P[:, c] + beta * Q[:, c], PANEL_ROWS rows per workgroup.
// Bound by reading X once (n^2 elements per product).  X is symmetric, so rows of
// X are read as columns: 16-byte loads contiguous in k.  The X tile is staged in
// LDS as FP32 [k][row] and each thread accumulates a 4 x 4 block (4 rows, 4 of
// the m <= 32 columns), i.e. two 16-byte LDS reads per 16 FMAs.
constexpr int PANEL_ROWS = 128;
constexpr int PANEL_K = 64;

template <typename TI>
__device__ __forceinline__ void panel_load_x(const TI *__restrict__ X, int ld, int i0, int k0,
                                             float (*sX)[PANEL_ROWS + 4], bool kb) {
  constexpr int EPU = 16 / (int)sizeof(TI);                  // elements per 16-byte load
  constexpr int CPR = PANEL_K / EPU;                         // loads per row
  constexpr int PER_T = PANEL_ROWS * CPR / 256;
#pragma unroll
  for (int q = 0; q < PER_T; ++q) {
    const int idx = threadIdx.x + 256 * q, row = idx / CPR, kc = idx % CPR;
    uint4 v = {0u, 0u, 0u, 0u};
    if (i0 + row < ld)     // row i0 + row of X = its column (symmetric), k-blocked or not
      v = *reinterpret_cast<const uint4 *>(
          X + (kb ? kb_index(k0 + kc * EPU, i0 + row, ld) : (int64_t)(i0 + row) * ld + k0 + kc * EPU));
    const TI *e = reinterpret_cast<const TI *>(&v);
#pragma unroll
    for (int j = 0; j < EPU; ++j) sX[kc * EPU + j][row] = to_f32<TI>(e[j]);
  }
}

template <typename TI>
__device__ void panel_mul_body(const TI *__restrict__ X, const float *__restrict__ P,
                               const float *__restrict__ Q, float *__restrict__ O, int ld, int m,
                               float alpha, float beta, float (*sX)[PANEL_ROWS + 4],
                               float (*sP)[MAXM], bool kb) {
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * PANEL_ROWS;
  const int ti = tid & 31, tc = tid >> 5;         // rows 4 ti .. 4 ti + 3, columns 4 tc .. + 3
  float acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0f;
  for (int k0 = 0; k0 < ld; k0 += PANEL_K) {
    panel_load_x<TI>(X, ld, i0, k0, sX, kb);
    for (int e = tid; e < PANEL_K * MAXM; e += 256) {
      const int kk = e % PANEL_K, c = e / PANEL_K;
      sP[kk][c] = c < m ? P[(int64_t)c * ld + k0 + kk] : 0.0f;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < PANEL_K; ++kk) {
      const float4 x = *reinterpret_cast<const float4 *>(&sX[kk][4 * ti]);
      const float4 p = *reinterpret_cast<const float4 *>(&sP[kk][4 * tc]);
      const float xs[4] = {x.x, x.y, x.z, x.w}, ps[4] = {p.x, p.y, p.z, p.w};
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] += xs[r] * ps[c];
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int col = 4 * tc + c;
    if (col >= m) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + 4 * ti + r;
      if (i >= ld) continue;
      float v = alpha * acc[r][c];
      if (beta != 0.0f) v += beta * Q[(int64_t)col * ld + i];
      O[(int64_t)col * ld + i] = v;
    }
  }
}

// FP32 and BF16 iterates (FP16 ones go to panel_mfma_kernel).
__global__ __launch_bounds__(256) void panel_mul_kernel(const SubDesc *__restrict__ desc,
                                                        const SubState *__restrict__ st, char *ws,
                                                        int qp, int qq, int qo, float alpha,
                                                        float beta) {
  const SubDesc d = desc[blockIdx.y];
  const SubState &s = st[blockIdx.y];
  if (s.status != 0 || s.prec == P_FP16 || blockIdx.x * PANEL_ROWS >= (unsigned)d.npad) return;
  const int c0 = MAXM * blockIdx.z;              // this workgroup's chunk of own columns
  if (c0 >= d.m) return;
  const int mc = d.m - c0 < MAXM ? d.m - c0 : MAXM;
  __shared__ float sX[PANEL_K][PANEL_ROWS + 4];
  __shared__ float sP[PANEL_K][MAXM];
  const int64_t co = (int64_t)c0 * d.npad;
  const float *P = panel_ptr(ws, d, qp) + co;
  const float *Q = panel_ptr(ws, d, qq) + co;
  float *O = panel_ptr(ws, d, qo) + co;
  const char *xb = ws + d.off_lo + (int64_t)s.cur * 4 * d.npad * d.npad;
  const bool kb = d.kb != 0;                     // BF16 here: k-blocked on the large tiles
  if (s.prec == P_FP32)
    panel_mul_body<float>(reinterpret_cast<const float *>(xb), P, Q, O, d.npad, mc, alpha, beta,
                          sX, sP, false);
  else if (s.prec == P_FP16)
    panel_mul_body<_Float16>(reinterpret_cast<const _Float16 *>(xb), P, Q, O, d.npad, mc, alpha,
                             beta, sX, sP, kb);
  else
    panel_mul_body<__bf16>(reinterpret_cast<const __bf16 *>(xb), P, Q, O, d.npad, mc, alpha,
                           beta, sX, sP, kb);
}

// O = alpha X P + beta Q for submatrices iterating in FP16, on MFMAs.  X is exactly
// FP16; P (FP32) is split as P = hi + 2^-11 lo with hi, lo FP16, so
//   X P = X hi + 2^-11 X lo,
// every term within 2^-22 of its exact value, sums in FP32 (two
// v_mfma_f32_32x32x16_f16 per 32 x 32 block and 16 k).  A wave owns PM_BLK blocks
// of 32 rows and all m <= 32 columns, so each B fragment (P, split in registers)
// serves PM_BLK row blocks; A fragments come straight from X (row i of X is column
// i, contiguous in k), B fragments from P (column c is contiguous in k).  Lane
// (h, c) supplies k = 8 h .. 8 h + 7 of its row (A) and of column c (B); the result
// D(r, c) of register q sits in lane c + 32 h with r = 8 (q / 4) + 4 h + q % 4.
typedef _Float16 ph8 __attribute__((ext_vector_type(8)));
typedef float pf16 __attribute__((ext_vector_type(16)));
constexpr float PANEL_LO_SCALE = 2048.0f;
constexpr int PM_BLK = 2;                         // 32-row blocks per wave
constexpr int PM_ROWS = 4 * 32 * PM_BLK;          // rows per workgroup

__global__ __launch_bounds__(256) void panel_mfma_kernel(const SubDesc *__restrict__ desc,
                                                         const SubState *__restrict__ st,
                                                         char *ws, int qp, int qq, int qo,
                                                         float alpha, float beta) {
  const SubDesc d = desc[blockIdx.y];
  const SubState &s = st[blockIdx.y];
  if (s.status != 0 || s.prec != P_FP16) return;
  const int c0 = MAXM * blockIdx.z;              // this workgroup's chunk of own columns
  if (c0 >= d.m) return;
  const int ld = d.npad, m = d.m - c0 < MAXM ? d.m - c0 : MAXM;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, h = lane >> 5, c = lane & 31;
  const int i0 = blockIdx.x * PM_ROWS + 32 * PM_BLK * w;
  if (i0 >= ld) return;                                   // the whole wave
  int nb = (ld - i0) / 32;                                // row blocks inside the matrix
  nb = nb > PM_BLK ? PM_BLK : nb;
  const _Float16 *X = reinterpret_cast<const _Float16 *>(ws + d.off_lo) +
                      (int64_t)s.cur * 2 * ld * ld;
  const int64_t co = (int64_t)c0 * ld;
  const float *P = panel_ptr(ws, d, qp) + co;
  const float *Q = panel_ptr(ws, d, qq) + co;
  float *O = panel_ptr(ws, d, qo) + co;
  const bool live = c < m;
  // row i of X (= its column) at k .. k + 7: k-blocked on the large tiles
  const bool kb = d.kb != 0;
  const _Float16 *xr = X + (int64_t)(i0 + c) * ld + 8 * h;
  const float *pc = P + (int64_t)(live ? c : 0) * ld + 8 * h;
  pf16 ah[PM_BLK], al[PM_BLK];
#pragma unroll
  for (int b = 0; b < PM_BLK; ++b)
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      ah[b][q] = 0.0f;
      al[b][q] = 0.0f;
    }
#pragma unroll 4
  for (int k = 0; k < ld; k += 16) {
    float4 p0 = {0.0f, 0.0f, 0.0f, 0.0f}, p1 = p0;
    if (live) {
      p0 = *reinterpret_cast<const float4 *>(pc + k);
      p1 = *reinterpret_cast<const float4 *>(pc + k + 4);
    }
    ph8 a[PM_BLK];
#pragma unroll
    for (int b = 0; b < PM_BLK; ++b)
      if (b < nb)
        a[b] = *reinterpret_cast<const ph8 *>(
            kb ? X + kb_index(k + 8 * h, i0 + c + 32 * b, ld) : xr + (int64_t)32 * b * ld + k);
    const float pv[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
    ph8 bh, bl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const _Float16 hi = (_Float16)pv[e];
      bh[e] = hi;
      bl[e] = (_Float16)((pv[e] - (float)hi) * PANEL_LO_SCALE);
    }
#pragma unroll
    for (int b = 0; b < PM_BLK; ++b)
      if (b < nb) {
        ah[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[b], bh, ah[b], 0, 0, 0);
        al[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[b], bl, al[b], 0, 0, 0);
      }
  }
  if (!live) return;
#pragma unroll
  for (int b = 0; b < PM_BLK; ++b) {
    if (b >= nb) continue;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = i0 + 32 * b + 8 * (q >> 2) + 4 * h + (q & 3);
      float v = alpha * (ah[b][q] + al[b][q] * (1.0f / PANEL_LO_SCALE));
      if (beta != 0.0f) v += beta * Q[(int64_t)c * ld + r];
      O[(int64_t)c * ld + r] = v;
    }
  }
}

// Dcol[i, c] = 1/2 sum_{k >= i} Linv[k, i] (V[k, c] - W[k, c]) in FP64 on
// v_mfma_f64_16x16x4_f64, straight from global memory (no LDS, no barriers): wave w
// owns rows i0 + 16 w .. + 15 of Dcol and the two 16-column blocks of the chunk.  The
// instruction takes A(i, k) from lane i + 16 k and B(k, c) from lane c + 16 k; the
// sum over k may run in any order that A and B share, so within each 32-row chunk
// of k, k slot j of step s is row k0 + 8 j + s: lane i + 16 j reads 8 consecutive
// rows of column i of L^-1 (64 contiguous bytes) and lane c + 16 j 8 rows of V and
// W.  The next chunk is loaded while the current one is multiplied.  D(i, c) sits
// in lane c + 16 (i % 4), register i / 4.
constexpr int DCOL_KC = 32;             // rows of k per chunk

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void dcol_kernel(const SubDesc *__restrict__ desc, const SubState *__restrict__ st, char *ws,
                 int qv, int qw) {
  const SubDesc d = desc[blockIdx.y];
  if (st[blockIdx.y].status != 0) return;
  const int c0 = MAXM * blockIdx.z;              // this workgroup's chunk of own columns
  if (c0 >= d.m) return;
  const int ld = d.npad, m = d.m - c0 < MAXM ? d.m - c0 : MAXM;
  const int i0 = blockIdx.x * 64;
  if (i0 >= ld) return;
  const int64_t co = (int64_t)c0 * ld;
  const double *Li = reinterpret_cast<const double *>(ws + d.off_s);
  const float *V = panel_ptr(ws, d, qv) + co;
  const float *W = panel_ptr(ws, d, qw) + co;
  double *Dc = reinterpret_cast<double *>(ws + d.off_dcol) + co;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kq = 8 * (lane >> 4);                // this lane's rows within a chunk
  // L^-1 is lower triangular: rows k < i0 of these columns are zero, so k starts at i0
  const double *Lc = Li + (int64_t)(i0 + 16 * w + (lane & 15)) * ld + kq;
  const float *Vc[2], *Wc[2];
  bool cin[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int c = 16 * t + (lane & 15);
    cin[t] = c < m;
    Vc[t] = V + (int64_t)(cin[t] ? c : 0) * ld + kq;
    Wc[t] = W + (int64_t)(cin[t] ? c : 0) * ld + kq;
  }
  typedef double d2 __attribute__((ext_vector_type(2)));
  double a[2][8], u[2][2][8];
  auto fetch = [&](int k0, int b) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const d2 v = *reinterpret_cast<const d2 *>(Lc + k0 + 2 * j);
      a[b][2 * j] = v.x;
      a[b][2 * j + 1] = v.y;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        float4 x = {0.0f, 0.0f, 0.0f, 0.0f}, y = x;
        if (cin[t]) {
          x = *reinterpret_cast<const float4 *>(Vc[t] + k0 + 4 * j);
          y = *reinterpret_cast<const float4 *>(Wc[t] + k0 + 4 * j);
        }
        u[b][t][4 * j] = (double)x.x - (double)y.x;
        u[b][t][4 * j + 1] = (double)x.y - (double)y.y;
        u[b][t][4 * j + 2] = (double)x.z - (double)y.z;
        u[b][t][4 * j + 3] = (double)x.w - (double)y.w;
      }
    }
  };
  d4 acc[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};
  auto mul = [&](int b) {
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
      for (int t = 0; t < 2; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[b][s2], u[b][t][s2], acc[t], 0, 0, 0);
  };
  fetch(i0, 0);
  int k0 = i0;
  for (; k0 + DCOL_KC < ld; k0 += 2 * DCOL_KC) {
    fetch(k0 + DCOL_KC, 1);
    mul(0);
    if (k0 + 2 * DCOL_KC < ld) fetch(k0 + 2 * DCOL_KC, 0);
    mul(1);
  }
  if (k0 < ld) mul(0);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int c = 16 * t + (lane & 15);
    if (c >= m) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      Dc[(int64_t)c * ld + i0 + 16 * w + 4 * q + (lane >> 4)] = 0.5 * acc[t][q];
  }
}

// Write the block columns of the submatrix's own molecules into D and sum their
// contributions to Tr(DH), Tr(DS).  For own molecule J, every stored block (I, J)
// of D takes rows of member I and J's own columns of T_k(D); member I is found by a
// binary search over the members in ascending molecule order (LDS).
constexpr int SCATTER_MAXMEM = 1024;

__global__ __launch_bounds__(256) void scatter_kernel(
    const SubDesc *__restrict__ desc, const SubState *__restrict__ st,
    const int32_t *__restrict__ mem_mol, const int32_t *__restrict__ mem_loc,
    const int32_t *__restrict__ mem_srt, const int32_t *__restrict__ blk_dim,
    const int64_t *__restrict__ colptr, const int32_t *__restrict__ rowblk,
    const int64_t *__restrict__ valoff, double *__restrict__ D_val,
    const double *__restrict__ H_val, const double *__restrict__ S_val, const char *ws,
    nolsm_stats *__restrict__ stats) {
  const SubDesc d = desc[blockIdx.x];
  __shared__ double red[4];
  __shared__ int32_t s_mol[SCATTER_MAXMEM];     // members in ascending molecule order
  __shared__ int32_t s_loc[SCATTER_MAXMEM];     // their first rows in T_k
  const double *Dc = reinterpret_cast<const double *>(ws + d.off_dcol);
  const bool ok = st[blockIdx.x].status == 0;
  for (int a = threadIdx.x; a < d.nmem; a += 256) {
    const int q = mem_srt[d.mem_off + a];
    s_mol[a] = mem_mol[d.mem_off + q];
    s_loc[a] = mem_loc[d.mem_off + q];
  }
  __syncthreads();
  double eh = 0.0, es = 0.0;
  for (int j = 0; j < d.ngrp; ++j) {
    const int J = mem_mol[d.mem_off + d.own_mem + j];
    const int col0 = mem_loc[d.mem_off + d.own_mem + j] - d.own_lo;   // J's first own column
    const int dJ = blk_dim[J];
    for (int64_t t = colptr[J]; t < colptr[J + 1]; ++t) {
      const int I = rowblk[t];
      int lo = 0, hi = d.nmem;                   // first member >= I (I is a member)
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_mol[mid] < I) lo = mid + 1; else hi = mid;
      }
      const int loc = s_loc[lo];
      const int dI = blk_dim[I];
      const int64_t base = valoff[t];
      for (int e = threadIdx.x; e < dI * dJ; e += 256) {
        const int c = e / dI, r = e - c * dI;
        const double v = ok ? Dc[(int64_t)(col0 + c) * d.npad + loc + r] : 0.0;
        D_val[base + e] = v;
        eh += v * H_val[base + e];
        es += v * S_val[base + e];
      }
    }
  }
  eh = block_sum256(eh, red);
  es = block_sum256(es, red);
  if (threadIdx.x == 0 && stats) {
    stats[blockIdx.x].tr_dh = eh;
    stats[blockIdx.x].tr_ds = es;
  }
}

__global__ __launch_bounds__(256) void coltrace_kernel(const int32_t *__restrict__ blk_dim,
                                                       const int64_t *__restrict__ colptr,
                                                       const int32_t *__restrict__ rowblk,
                                                       const int64_t *__restrict__ valoff,
                                                       const double *__restrict__ D_val,
                                                       const double *__restrict__ H_val,
                                                       const double *__restrict__ S_val,
                                                       double *__restrict__ col_traces) {
  const int k = blockIdx.x;
  __shared__ double red[4];
  double eh = 0.0, es = 0.0;
  const int dk = blk_dim[k];
  for (int64_t t = colptr[k]; t < colptr[k + 1]; ++t) {
    const int sz = blk_dim[rowblk[t]] * dk;
    const int64_t b = valoff[t];
    for (int e = threadIdx.x; e < sz; e += 256) {
      const double v = D_val[b + e];
      eh += v * H_val[b + e];
      es += v * S_val[b + e];
    }
  }
  eh = block_sum256(eh, red);
  es = block_sum256(es, red);
  if (threadIdx.x == 0) {
    col_traces[2 * k] = eh;
    col_traces[2 * k + 1] = es;
  }
}

__global__ __launch_bounds__(256) void final_trace_kernel(const double *__restrict__ col_traces,
                                                          int nmol, double *__restrict__ out2) {
  __shared__ double red[4];
  double eh = 0.0, es = 0.0;
  for (int k = threadIdx.x; k < nmol; k += 256) {
    eh += col_traces[2 * k];
    es += col_traces[2 * k + 1];
  }
  eh = block_sum256(eh, red);
  es = block_sum256(es, red);
  if (threadIdx.x == 0) {
    out2[0] = eh;
    out2[1] = es;
  }
}

// Copy the per-submatrix record to the caller's stats array.
__global__ void stats_kernel(const SubDesc *__restrict__ desc, const SubState *__restrict__ st,
                             int K, nolsm_stats *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const SubState &s = st[i];
  nolsm_stats r;
  r.n = desc[i].n;
  r.status = s.status;
  r.iters_lo = s.iters_lo;
  r.iters_fb = s.iters_fb;
  r.resid = s.resid;
  r.fell_back = s.fell_back;
  r.scale = s.scale;
  r.tr_dh = 0.0;
  r.tr_ds = 0.0;
  r.tr_x = s.tr_x;
  r.n_neg = (int32_t)lrintf(0.5f * ((float)r.n - s.tr_x));
  out[i] = r;
}

// Tr(X) of every submatrix's final iterate, in its storage precision summed in FP32
// (fixed order: one workgroup per submatrix).
__global__ __launch_bounds__(256) void trace_x_kernel(const SubDesc *__restrict__ desc,
                                                      SubState *__restrict__ st,
                                                      const char *ws) {
  const SubDesc d = desc[blockIdx.x];
  SubState &s = st[blockIdx.x];
  __shared__ float red[4];
  const char *xb = ws + d.off_lo + (int64_t)s.cur * 4 * d.npad * d.npad;
  const bool kb = d.kb && s.prec != P_FP32;                // k-blocked FP16/BF16 iterate
  float t = 0.0f;
  for (int i = threadIdx.x; i < d.n; i += 256) {
    const int64_t o = kb ? kb_index(i, i, d.npad) : (int64_t)i * d.npad + i;
    if (s.prec == P_FP32) t += reinterpret_cast<const float *>(xb)[o];
    else if (s.prec == P_FP16) t += (float)reinterpret_cast<const _Float16 *>(xb)[o];
    else t += (float)reinterpret_cast<const __bf16 *>(xb)[o];
  }
  t = block_sum256(t, red);
  if (threadIdx.x == 0) s.tr_x = s.status == 0 ? t : 0.0f;
}

// ------------------------------------------------------------------ host side

__global__ __launch_bounds__(256) void panel_axpby_kernel(const SubDesc *__restrict__ desc,
                                                          const SubState *__restrict__ st,
                                                          char *ws, int qa, int qb, float alpha,
                                                          float beta) {
  const SubDesc d = desc[blockIdx.y];
  if (st[blockIdx.y].status != 0) return;
  float *A = panel_ptr(ws, d, qa);
  const float *B = panel_ptr(ws, d, qb);
  const int total = d.npad * d.m;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256)
    A[e] = alpha * A[e] + beta * B[e];
}

// g_s(P) = F_s P with F_0 = X, F_s = f(F_{s-1}), f(X) = 1/2 X (3I - X^2):
//   g_0(P) = X P,   g_s(P) = 3/2 g_{s-1}(P) - 1/2 g_{s-1}(g_{s-1}(g_{s-1}(P))).
// 3^s panel products.  Slots are panel buffers; returns the slot holding g_s(P).
struct PanelCtx {
  const SubDesc *desc;
  const SubState *st;
  int K, max_npad, nchunk;
  char *ws;
  hipStream_t s;
  unsigned used;
  int alloc() {
    for (int q = 0; q < NPANEL; ++q)
      if (!(used & (1u << q))) { used |= 1u << q; return q; }
    return -1;
  }
  void release(int q) { used &= ~(1u << q); }
  int apply(int steps, int qin) {
    const dim3 grid((max_npad + PANEL_ROWS - 1) / PANEL_ROWS, K, nchunk);
    if (steps == 0) {
      const int qo = alloc();
      panel_mfma_kernel<<<dim3((max_npad + PM_ROWS - 1) / PM_ROWS, K, nchunk), 256, 0, s>>>(
          desc, st, ws, qin, qin, qo, 1.0f, 0.0f);
      panel_mul_kernel<<<grid, 256, 0, s>>>(desc, st, ws, qin, qin, qo, 1.0f, 0.0f);
      return qo;
    }
    const int q1 = apply(steps - 1, qin);
    const int q2 = apply(steps - 1, q1);
    const int q3 = apply(steps - 1, q2);
    release(q2);
    panel_axpby_kernel<<<dim3(64, K), 256, 0, s>>>(desc, st, ws, q1, q3, 1.5f, -0.5f);
    release(q3);
    return q1;
  }
};

void launch_lit_panel_v(const SubDesc *desc, const SubState *st, int K, char *ws, int qv,
                        hipStream_t s);
void launch_lit_dcol(const SubDesc *desc, const SubState *st, int K, char *ws, int qv, int qw,
                     hipStream_t s);

// literal: V = S^-1[:, own] and T_k(D)[:, own] = 1/2 (V - W) (literal.hip)
void launch_density_columns(const SubDesc *desc, const SubState *st, int K, int max_npad,
                            int max_m, char *ws, int panel_steps, bool literal, hipStream_t s) {
  const int nchunk = (max_m + MAXM - 1) / MAXM;   // own columns in chunks of MAXM
  PanelCtx c{desc, st, K, max_npad, nchunk, ws, s, 1u};   // slot 0 holds V
  if (literal) launch_lit_panel_v(desc, st, K, ws, 0, s);
  else panel_v_kernel<<<dim3(64, K), 256, 0, s>>>(desc, st, ws, 0);
  const int qw = c.apply(panel_steps, 0);
  if (literal) launch_lit_dcol(desc, st, K, ws, 0, qw, s);
  else dcol_kernel<<<dim3(max_npad / 64, K, nchunk), 256, 0, s>>>(desc, st, ws, 0, qw);
}

void launch_scatter(const SubDesc *desc, const SubState *st, int K, int maxmem,
                    const int32_t *mem_mol, const int32_t *mem_loc, const int32_t *mem_srt,
                    const nolsm_pattern *pat, double *D_val, const double *H_val,
                    const double *S_val, const char *ws, nolsm_stats *stats, hipStream_t s) {
  (void)maxmem;                  // plans keep at most SCATTER_MAXMEM members per submatrix
  scatter_kernel<<<K, 256, 0, s>>>(desc, st, mem_mol, mem_loc, mem_srt, pat->blk_dim,
                                   pat->colptr, pat->rowblk, pat->valoff, D_val, H_val, S_val,
                                   ws, stats);
}

void launch_energy(const nolsm_pattern *pat, int nmol, const double *D_val, const double *H_val,
                   const double *S_val, double *col_traces, double *out2, hipStream_t s) {
  coltrace_kernel<<<nmol, 256, 0, s>>>(pat->blk_dim, pat->colptr, pat->rowblk, pat->valoff,
                                       D_val, H_val, S_val, col_traces);
  final_trace_kernel<<<1, 256, 0, s>>>(col_traces, nmol, out2);
}

// Per-block-column partial traces for callers that cannot allocate (graph capture,
// serving loops): a fixed array in device memory, one copy per GPU, shared by every
// such call on that GPU.  coltrace_kernel writes every entry it covers before
// final_trace_kernel reads it, so nothing needs clearing between calls.
static __device__ __align__(256) double scratch[2 * ENERGY_NOALLOC_MAXMOL];

// Device address of `scratch` on the current device, looked up once per device.
hipError_t energy_scratch_ptr(double **out) {
  static std::mutex mtx;
  static double *ptrs[MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mtx);
  if (!ptrs[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptrs[dev] = static_cast<double *>(p);
  }
  *out = ptrs[dev];
  return hipSuccess;
}

void launch_trace_x(const SubDesc *desc, SubState *st, int K, const char *ws, hipStream_t s) {
  trace_x_kernel<<<K, 256, 0, s>>>(desc, st, ws);
}

void launch_stats(const SubDesc *desc, const SubState *st, int K, nolsm_stats *out,
                  hipStream_t s) {
  stats_kernel<<<(K + 255) / 256, 256, 0, s>>>(desc, st, K, out);
}

}  // namespace nolsm
