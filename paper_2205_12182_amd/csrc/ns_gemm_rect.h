// Sign-iteration product for large submatrices: 256 x 128 tiles, two workgroups
// per CU (paper, Eq. 6; same contraction and epilogue semantics as ns_gemm_body).
//
// The 256 x 256 tile of ns_gemm_body needs all 512 registers of a SIMD lane for
// its accumulators, so only one workgroup fits per CU and the tile's loads and
// its epilogue stores (the new iterate, written once in each triangle) cannot
// overlap with MFMAs.  Here a wave owns a 128 x 64 block (4 x 2 blocks of
// 32 x 32, 128 accumulator registers), a workgroup of four waves a 256 x 128
// tile, and the LDS ring has three slots of 24 KiB, so two workgroups are
// resident per CU and one's memory phases run under the other's MFMAs.
//
// Stages are loaded straight into LDS (buffer loads with the LDS destination),
// two stages ahead; rows are 64 bytes with the conflict-free chunk permutation.
// The epilogue stores from registers: 8-byte stores of four consecutive rows of
// a column for the tile itself and 2-byte stores for its mirror image.
#pragma once
#include "ns_gemm.h"

namespace nolsm {

constexpr int RT_M = 256, RT_N = 128;                 // tile rows x columns
constexpr int RT_SLOT_U4 = (RT_M + RT_N) * 4;          // one ring slot: A rows, then B rows

template <typename TI, int EPI, bool PARTIAL>
__device__ __forceinline__ void ns_gemm_rect_body(const TI *__restrict__ A,
                                                  const TI *__restrict__ B, TI *__restrict__ Out,
                                                  int ld, int n, int i0, int j0, float c1,
                                                  float c3, uint4 *s0, uint4 *s1, uint4 *s2,
                                                  float *red, unsigned long long *racc) {
  constexpr int BM = 4, BN = 2;                        // 32 x 32 blocks per wave
  constexpr int LA = RT_M / 64, LB = RT_N / 64;        // loads per wave per stage (A, B)
  constexpr int LPS = LA + LB;
  constexpr int BOFF = RT_M * 4;                       // first B row in a slot (uint4)
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (w >> 1) * 32 * BM, wn = (w & 1) * 32 * BN;
  const int h = lane >> 5, l32 = lane & 31;
  const int nk = ld / KStage<TI>::KS;

  int nvr = BM, nvc = BN;
  if (PARTIAL) {
    nvr = (ld - i0 - wm) / 32;
    nvc = (ld - j0 - wn) / 32;
    nvr = nvr < 0 ? 0 : (nvr > BM ? BM : nvr);
    nvc = nvc < 0 ? 0 : (nvc > BN ? BN : nvc);
  }

  // rows past npad (ragged edge tiles) read as zero; stages past the last one are
  // issued against zero-size resources so every wave issues the same loads
  const int nrec = ld * ld * (int)sizeof(TI);
  const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(A), (short)0, nrec, BUFFER_RSRC_WORD3);
  const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(B), (short)0, nrec, BUFFER_RSRC_WORD3);
  const __amdgpu_buffer_rsrc_t rA0 = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(A), (short)0, 0, BUFFER_RSRC_WORD3);
  const __amdgpu_buffer_rsrc_t rB0 = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(B), (short)0, 0, BUFFER_RSRC_WORD3);

  // load q of a wave fills rows 16 (4 q + w) .. + 15 of its panel (see ns_gemm_body)
  unsigned voA[LA], voB[LB];
#pragma unroll
  for (int q = 0; q < LA; ++q) {
    const int row = 16 * (4 * q + w) + (lane >> 2);
    const unsigned ch = (unsigned)((lane & 3) ^ chunk_swz(row));
    voA[q] = (unsigned)((i0 + row) * ld) * (unsigned)sizeof(TI) + 16u * ch;
  }
#pragma unroll
  for (int q = 0; q < LB; ++q) {
    const int row = 16 * (4 * q + w) + (lane >> 2);
    const unsigned ch = (unsigned)((lane & 3) ^ chunk_swz(row));
    voB[q] = (unsigned)((j0 + row) * ld) * (unsigned)sizeof(TI) + 16u * ch;
  }
  const int z = chunk_swz(l32);
  const int fa0 = (wm + l32) * 4 + ((2 * h) ^ z), fa1 = (wm + l32) * 4 + ((2 * h + 1) ^ z);
  const int fb0 = BOFF + (wn + l32) * 4 + ((2 * h) ^ z),
            fb1 = BOFF + (wn + l32) * 4 + ((2 * h + 1) ^ z);

  f16x acc[BM][BN];
#pragma unroll
  for (int bm = 0; bm < BM; ++bm)
#pragma unroll
    for (int bn = 0; bn < BN; ++bn)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[bm][bn][q] = 0.0f;

  auto issue = [&](uint4 *slot, int kt) {
    const bool live = kt < nk;
    const __amdgpu_buffer_rsrc_t ra = live ? rA : rA0, rb = live ? rB : rB0;
    const int so = live ? 64 * kt : 0;
#pragma unroll
    for (int q = 0; q < LA; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, NS_LDS_PTR(slot + (4 * q + w) * 64), 16,
                                               voA[q], so, 0, 0);
#pragma unroll
    for (int q = 0; q < LB; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, NS_LDS_PTR(slot + BOFF + (4 * q + w) * 64),
                                               16, voB[q], so, 0, 0);
  };
  // Step kt: stage kt has landed once only stage kt + 1 is still in flight; after
  // the barrier every wave is done with the slot of stage kt - 1, which takes
  // stage kt + 2.  Fragments are read and consumed within the step; the other
  // workgroup on the CU covers the LDS latency.
  constexpr int NDS = 2 * (BM + BN), NMF = BM * BN * Mfma<TI>::STEPS;
  auto step = [&](const uint4 *cur, uint4 *refill, int kt) {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(LPS));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    uint4 af[BM][2], bf[BN][2];
#pragma unroll
    for (int b = 0; b < BM; ++b) {
      af[b][0] = cur[fa0 + 128 * b];
      af[b][1] = cur[fa1 + 128 * b];
    }
#pragma unroll
    for (int b = 0; b < BN; ++b) {
      bf[b][0] = cur[fb0 + 128 * b];
      bf[b][1] = cur[fb1 + 128 * b];
    }
    issue(refill, kt + 2);
#pragma unroll
    for (int s = 0; s < Mfma<TI>::STEPS; ++s)
#pragma unroll
      for (int bm = 0; bm < BM; ++bm)
#pragma unroll
        for (int bn = 0; bn < BN; ++bn)
          if (!PARTIAL || (bm < nvr && bn < nvc))
            acc[bm][bn] = Mfma<TI>::op(af[bm], bf[bn], s, acc[bm][bn]);
    if (!PARTIAL) {
      __builtin_amdgcn_sched_group_barrier(0x100, NDS, 0);                 // LDS reads
#pragma unroll
      for (int j = 0; j < LPS; ++j) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);                // MFMA
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);                // memory load
      }
      __builtin_amdgcn_sched_group_barrier(0x008, NMF - 2 * LPS, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  };

  issue(s0, 0);
  issue(s1, 1);
  int kt = 0;
  for (; kt + 3 <= nk; kt += 3) {
    step(s0, s2, kt);
    step(s1, s0, kt + 1);
    step(s2, s1, kt + 2);
  }
  if (nk - kt > 0) step(s0, s2, kt);
  if (nk - kt > 1) step(s1, s0, kt + 1);
  // the trailing (empty) loads target LDS: drain them before the workgroup ends
  __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));

  // Epilogue from registers.  Element (r, c) of block (bm, bn), register q:
  //   r = wm + 32 bm + 8 (q >> 2) + 4 h + (q & 3),  c = wn + 32 bn + l32.
  // Only r <= c (global) is kept; (r, c) goes to Out[c ld + r] and, for r < c, the
  // mirror (c, r) to Out[r ld + c].  SQUARE turns X^2 into Z = c1 I + c3 X^2 and
  // accumulates the residual ||X^2 - I||_F^2 from X^2.
  const bool cross = (i0 < j0 + RT_N) && (j0 < i0 + RT_M);    // tile meets the diagonal
  int ldv = ld;
  asm volatile("" : "+v"(ldv));
  float rs = 0.0f;     // crossing tiles: weighted sum; other tiles: plain sum (weight 2 later)
#pragma unroll
  for (int bm = 0; bm < BM; ++bm)
#pragma unroll
    for (int bn = 0; bn < BN; ++bn) {
      if (PARTIAL && (bm >= nvr || bn >= nvc)) continue;
      const int c = wn + 32 * bn + l32, gc = j0 + c;
      TI *col = Out + (int64_t)gc * ldv + i0;
      TI *mir = Out + (int64_t)(i0 + wm + 32 * bm + 4 * h) * ldv + gc;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int r0 = wm + 32 * bm + 8 * g + 4 * h;
        if (!cross) {                                     // every element has r < c
          typedef TI v4 __attribute__((ext_vector_type(4)));
          v4 ov;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            float v = acc[bm][bn][4 * g + e];
            if (EPI == EPI_SQUARE) {
              rs += v * v;
              v = c3 * v;
            }
            ov[e] = from_f32<TI>(v);
            mir[(int64_t)(8 * g + e) * ldv] = ov[e];
          }
          *reinterpret_cast<v4 *>(col + r0) = ov;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int gr = i0 + r0 + e;
            float v = acc[bm][bn][4 * g + e];
            if (EPI == EPI_SQUARE) {
              const bool diag = gr == gc && gc < n;
              if (gr <= gc && gc < n) {
                const float df = v - (diag ? 1.0f : 0.0f);
                rs += (diag ? 1.0f : 2.0f) * df * df;
              }
              v = c3 * v + (diag ? c1 : 0.0f);
            }
            const TI o = from_f32<TI>(v);
            if (gr <= gc) col[r0 + e] = o;
            if (gr < gc) mir[(int64_t)(8 * g + e) * ldv] = o;
          }
        }
      }
    }
  if (EPI == EPI_SQUARE) {
    // tiles off the diagonal count each element twice (it stands for (r, c) and
    // (c, r)); padding rows and columns are zero and contribute nothing
    const float tot = block_sum256(cross ? rs : 2.0f * rs, red);
    if (tid == 0) atomicAdd(racc, resid_fixed(tot));
  }
}

// SQUARE: Z = c1 I + c3 X X (+ residual of X X);  UPDATE: X' = X Z.  Tiles are
// (256 ti, 128 tj) blocks of the upper triangle (2 ti <= tj).
template <typename TI, int EPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void ns_gemm_rect_kernel(const Tile *__restrict__ tiles, const SubDesc *__restrict__ desc,
                         SubState *__restrict__ st, char *ws, int prec,
                         unsigned long long *__restrict__ flop_units) {
  const Tile t = tiles[xcd_remap(blockIdx.x, gridDim.x)];
  SubState &S = st[t.sub];
  if (!S.active || S.prec != prec) return;
  const SubDesc d = desc[t.sub];
  const int ld = d.npad;
  const int cur = S.cur;
  const TI *A = buf_ptr<TI>(ws, d, cur);
  const TI *B = (EPI == EPI_SQUARE) ? A : buf_ptr<TI>(ws, d, (cur + 1) % 3);
  TI *Out = buf_ptr<TI>(ws, d, (cur + (EPI == EPI_SQUARE ? 1 : 2)) % 3);
  const int i0 = t.ti * RT_M, j0 = t.tj * RT_N;
  if (threadIdx.x == 0) {
    const int rows = (ld - i0 < RT_M ? ld - i0 : RT_M), cols = (ld - j0 < RT_N ? ld - j0 : RT_N);
    atomicAdd(flop_units, (unsigned long long)((rows / 32) * (cols / 32) * (ld / 64)));
  }
  __shared__ uint4 s0[RT_SLOT_U4], s1[RT_SLOT_U4], s2[RT_SLOT_U4];
  __shared__ float red[4];
  if (i0 + RT_M <= ld && j0 + RT_N <= ld)
    ns_gemm_rect_body<TI, EPI, false>(A, B, Out, ld, d.n, i0, j0, S.c1, S.c3, s0, s1, s2, red,
                                      &S.racc);
  else
    ns_gemm_rect_body<TI, EPI, true>(A, B, Out, ld, d.n, i0, j0, S.c1, S.c3, s0, s1, s2, red,
                                     &S.racc);
}

}  // namespace nolsm
