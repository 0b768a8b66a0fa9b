// Sign-iteration product for large submatrices: 256 x 128 tiles, two workgroups
// per CU (paper, Eq. 6; same contraction and epilogue semantics as ns_gemm_body).
//
// The 256 x 256 tile of ns_gemm_body needs all 512 registers of a SIMD lane for
// its accumulators, so only one workgroup fits per CU and the tile's loads and
// its epilogue stores (the new iterate, written once in each triangle) cannot
// overlap with MFMAs.  Here a wave owns a 128 x 64 block (8 x 4 blocks of 16 x 16,
// v_mfma_f32_16x16x32_f16/bf16, 128 accumulator registers), a workgroup of four
// waves a 256 x 128 tile, and the LDS ring has three slots of 24 KiB, so two
// workgroups are resident per CU and one's memory phases run under the other's
// MFMAs.  (The 16 x 16 x 32 MFMA covers a whole 32-k stage per instruction and
// issues faster than 32 x 32 x 16: measured 3% more throughput for this kernel.)
//
// The iterate is k-blocked (kb_index, common.h): a stage of 256 (or 128) columns is
// one contiguous block, loaded straight into LDS (buffer loads with the LDS
// destination), two stages ahead; rows are 64 bytes with the chunk permutation.
// (Measured against the column-major layout, whose stage rows are 64-byte runs one
// column apart: 7-10% less time per product.)
// Lane (g, l) of a fragment read takes chunk g (k = 8 g .. 8 g + 7) of row l of a
// 16-row block, for A and B alike.  The epilogue stores from registers: 8-byte
// stores of four consecutive rows of a column for the tile itself and, on tiles
// that meet the diagonal or the ragged edge, 2-byte stores for its mirror image.
#pragma once
#include "ns_gemm.h"

namespace nolsm {

constexpr int RT_M = 256, RT_N = 128;                 // tile rows x columns
constexpr int RT_SLOT_U4 = (RT_M + RT_N) * 4;          // one ring slot: A rows, then B rows

template <typename TI> struct Mfma16;
template <> struct Mfma16<_Float16> {
  __device__ static __forceinline__ f4x op(uint4 a, uint4 b, f4x c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a),
                                                  __builtin_bit_cast(h8, b), c, 0, 0, 0);
  }
};
template <> struct Mfma16<__bf16> {
  __device__ static __forceinline__ f4x op(uint4 a, uint4 b, f4x c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a),
                                                   __builtin_bit_cast(b8, b), c, 0, 0, 0);
  }
};

template <typename TI, int EPI, bool PARTIAL, bool LOWIDLE>
__device__ __forceinline__ void ns_gemm_rect_body(const TI *__restrict__ A,
                                                  const TI *__restrict__ B, TI *__restrict__ Out,
                                                  int ld, int n, int i0, int j0, float c1,
                                                  float c3, uint4 *s0, uint4 *s1, uint4 *s2,
                                                  float *red, unsigned long long *racc) {
  constexpr int BM = 8, BN = 4;                        // 16 x 16 blocks per wave
  constexpr int LA = RT_M / 64, LB = RT_N / 64;
  constexpr int LPS = LA + LB;
  constexpr int BOFF = RT_M * 4;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (w >> 1) * 128, wn = (w & 1) * 64;
  const int g = lane >> 4, l16 = lane & 15;
  const int nk = ld / KStage<TI>::KS;

  int nvr = BM, nvc = BN;
  // PARTIAL tiles are ragged at the matrix edge: blocks past the edge, and blocks
  // wholly below the diagonal (first row after last column), issue no MFMAs.
  // LOWIDLE tiles start on the diagonal (i0 == j0), so their second 128 rows lie
  // wholly below it: the two waves that own them issue no MFMAs, and those rows are
  // not loaded (the null buffer resource returns zeros without a memory access, so
  // every stage still issues the same number of loads).
  int diag_off = 0;                                   // row - column offset of block (0, 0)
  const bool skip_low = (PARTIAL || LOWIDLE) && i0 >= j0;
  const bool mfma_wave = !(LOWIDLE && wm >= 128);
  if (PARTIAL) {
    nvr = (ld - i0 - wm) / 16;
    nvc = (ld - j0 - wn) / 16;
    nvr = nvr < 0 ? 0 : (nvr > BM ? BM : nvr);
    nvc = nvc < 0 ? 0 : (nvc > BN ? BN : nvc);
    diag_off = (i0 + wm) - (j0 + wn);
  }
  const int nrec = ld * ld * (int)sizeof(TI);
  // k-blocked offsets: row r of a panel (column r of the iterate) starts at 64 r within
  // a stage's block, stage kt at 64 ld kt; rows past ld (the ragged edge) get an
  // offset past the buffer, which reads as zero
  constexpr unsigned KB_OOB = 0x80000000u;
  const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(A), (short)0, nrec, BUFFER_RSRC_WORD3);
  const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(B), (short)0, nrec, BUFFER_RSRC_WORD3);
  const __amdgpu_buffer_rsrc_t rA0 = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(A), (short)0, 0, BUFFER_RSRC_WORD3);
  const __amdgpu_buffer_rsrc_t rB0 = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(B), (short)0, 0, BUFFER_RSRC_WORD3);
  unsigned voA[LA], voB[LB];
#pragma unroll
  for (int q = 0; q < LA; ++q) {
    const int row = 16 * (4 * q + w) + (lane >> 2);
    const unsigned ch = (unsigned)((lane & 3) ^ chunk_swz(row));
    voA[q] = i0 + row < ld ? (unsigned)(i0 + row) * 64u + 16u * ch : KB_OOB;
  }
#pragma unroll
  for (int q = 0; q < LB; ++q) {
    const int row = 16 * (4 * q + w) + (lane >> 2);
    const unsigned ch = (unsigned)((lane & 3) ^ chunk_swz(row));
    voB[q] = j0 + row < ld ? (unsigned)(j0 + row) * 64u + 16u * ch : KB_OOB;
  }
  // lane (g, l16) reads chunk g of row l16 of each 16-row block (rows 16 b + l16 have
  // the same permutation for every b since 16 b does not change (r ^ (r >> 2)) & 3)
  const int z = chunk_swz(l16);
  const int fa = (wm + l16) * 4 + (g ^ z), fb = BOFF + (wn + l16) * 4 + (g ^ z);

  f4x acc[BM][BN];
#pragma unroll
  for (int bm = 0; bm < BM; ++bm)
#pragma unroll
    for (int bn = 0; bn < BN; ++bn)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[bm][bn][q] = 0.0f;

  auto issue = [&](uint4 *slot, int kt) {
    const bool live = kt < nk;
    const __amdgpu_buffer_rsrc_t ra = live ? rA : rA0, rb = live ? rB : rB0;
    const int so = live ? 64 * ld * kt : 0;
#pragma unroll
    for (int q = 0; q < LA; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds((skip_low && q >= LA / 2) ? rA0 : ra,
                                               NS_LDS_PTR(slot + (4 * q + w) * 64), 16,
                                               voA[q], so, 0, 0);
#pragma unroll
    for (int q = 0; q < LB; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, NS_LDS_PTR(slot + BOFF + (4 * q + w) * 64),
                                               16, voB[q], so, 0, 0);
  };
  constexpr int NDS = BM + BN, NMF = BM * BN;
  auto step = [&](const uint4 *cur, uint4 *refill, int kt) {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(LPS));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    if (LOWIDLE && !mfma_wave) {          // loads only; the same barriers as the others
      issue(refill, kt + 2);
      __builtin_amdgcn_sched_barrier(0);
      return;
    }
    uint4 af[BM], bf[BN];
#pragma unroll
    for (int b = 0; b < BM; ++b) af[b] = cur[fa + 64 * b];
#pragma unroll
    for (int b = 0; b < BN; ++b) bf[b] = cur[fb + 64 * b];
    issue(refill, kt + 2);
#pragma unroll
    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < BN; ++bn)
        if (!PARTIAL || (bm < nvr && bn < nvc && diag_off + 16 * (bm - bn) <= 15))
          acc[bm][bn] = Mfma16<TI>::op(af[bm], bf[bn], acc[bm][bn]);
    if (!PARTIAL) {
      __builtin_amdgcn_sched_group_barrier(0x100, NDS, 0);                 // LDS reads
#pragma unroll
      for (int j = 0; j < LPS; ++j) {
        __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);                // MFMA
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);                // memory load
      }
      __builtin_amdgcn_sched_group_barrier(0x008, NMF - 4 * LPS, 0);
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
  __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));

  // Epilogue: element (r, c) of block (bm, bn), register q:
  //   r = wm + 16 bm + 4 g + q,  c = wn + 16 bn + l16.
  const bool cross = (i0 < j0 + RT_N) && (j0 < i0 + RT_M);
  int ldv = ld;
  asm volatile("" : "+v"(ldv));
  float rs = 0.0f;
  typedef TI v4 __attribute__((ext_vector_type(4)));
  if (!PARTIAL && !LOWIDLE && !cross) {
    // Tiles off the diagonal: the tile's own columns are stored from registers (four
    // rows per lane); its mirror image goes through LDS.  Each wave stages its
    // 128 x 64 block in two halves of 64 rows, row-major (64 values + 8 of padding
    // per row), in the now idle ring (waves 0, 1 in slot 0, waves 2, 3 in slot 1),
    // and reads back 16-byte runs of a row: a row of the block is a 128-byte run of
    // one column of the mirror image, so the mirror is written in whole lines.
    // Only the wave that wrote a half reads it, so wave-local ordering suffices.
    constexpr int SLD = 72;
    constexpr int LGKM0 = 0xF | (0x3 << 14) | (0x7 << 4);   // lgkmcnt(0) only
    __syncthreads();                                        // the ring is free
    TI *stg = reinterpret_cast<TI *>(w < 2 ? s0 : s1) + (w & 1) * 64 * SLD;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int bm = 4 * h + b;
#pragma unroll
        for (int bn = 0; bn < BN; ++bn) {
          const int gc = j0 + wn + 16 * bn + l16;
          const int r0 = wm + 16 * bm + 4 * g;
          v4 ov;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            float v = acc[bm][bn][e];
            if (EPI == EPI_SQUARE) {
              rs += v * v;
              v = c3 * v;
            }
            ov[e] = from_f32<TI>(v);
            stg[(16 * b + 4 * g + e) * SLD + 16 * bn + l16] = ov[e];
          }
          *reinterpret_cast<v4 *>(Out + kb_index(i0 + r0, gc, ldv)) = ov;
        }
      }
      __builtin_amdgcn_s_waitcnt(LGKM0);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int e = lane + 64 * it, rr = e >> 3, ch = e & 7;
        const uint4 v = *reinterpret_cast<const uint4 *>(stg + rr * SLD + 8 * ch);
        *reinterpret_cast<uint4 *>(Out + kb_index(j0 + wn + 8 * ch, i0 + wm + 64 * h + rr,
                                                  ldv)) = v;
      }
      __builtin_amdgcn_s_waitcnt(LGKM0);
      __builtin_amdgcn_wave_barrier();
    }
    if (EPI == EPI_SQUARE) {
      const float tot = block_sum256(2.0f * rs, red);
      if (tid == 0) atomicAdd(racc, resid_fixed(tot));
    }
    return;
  }
#pragma unroll
  for (int bm = 0; bm < BM; ++bm)
#pragma unroll
    for (int bn = 0; bn < BN; ++bn) {
      if (PARTIAL && (bm >= nvr || bn >= nvc)) continue;
      const int c = wn + 16 * bn + l16, gc = j0 + c;
      const int r0 = wm + 16 * bm + 4 * g;
      // element (i0 + r0 + e, gc) and its mirror (gc, i0 + r0 + e)
      TI *col = Out + kb_index(i0 + r0, gc, ldv);
      TI *mir = Out + kb_index(gc, i0 + r0, ldv);
      if (!cross) {
        v4 ov;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float v = acc[bm][bn][e];
          if (EPI == EPI_SQUARE) {
            rs += v * v;
            v = c3 * v;
          }
          ov[e] = from_f32<TI>(v);
          mir[32 * e] = ov[e];
        }
        *reinterpret_cast<v4 *>(col) = ov;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int gr = i0 + r0 + e;
          float v = acc[bm][bn][e];
          if (EPI == EPI_SQUARE) {
            const bool diag = gr == gc && gc < n;
            if (gr <= gc && gc < n) {
              const float df = v - (diag ? 1.0f : 0.0f);
              rs += (diag ? 1.0f : 2.0f) * df * df;
            }
            v = c3 * v + (diag ? c1 : 0.0f);
          }
          const TI o = from_f32<TI>(v);
          if (gr <= gc) col[e] = o;
          if (gr < gc) mir[32 * e] = o;
        }
      }
    }
  if (EPI == EPI_SQUARE) {
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
    // the 16 x 16 blocks the four waves execute (ns_gemm_rect_body's predicates)
    const bool full = i0 + RT_M <= ld && j0 + RT_N <= ld;
    unsigned blocks = 0;
    for (int w = 0; w < 4; ++w) {
      const int wm = (w >> 1) * 128, wn = (w & 1) * 64;
      if (full) {
        blocks += (i0 == j0 && wm >= 128) ? 0u : 32u;
        continue;
      }
      int nvr = (ld - i0 - wm) / 16, nvc = (ld - j0 - wn) / 16;
      nvr = nvr < 0 ? 0 : (nvr > 8 ? 8 : nvr);
      nvc = nvc < 0 ? 0 : (nvc > 4 ? 4 : nvc);
      const int off = (i0 + wm) - (j0 + wn);
      for (int bm = 0; bm < nvr; ++bm)
        for (int bn = 0; bn < nvc; ++bn) blocks += (off + 16 * (bm - bn) <= 15) ? 1u : 0u;
    }
    atomicAdd(flop_units, (unsigned long long)blocks * (unsigned long long)(ld / 64));
  }
  __shared__ uint4 s0[RT_SLOT_U4], s1[RT_SLOT_U4], s2[RT_SLOT_U4];
  __shared__ float red[4];
  const bool full = i0 + RT_M <= ld && j0 + RT_N <= ld;
  if (full && i0 != j0)
    ns_gemm_rect_body<TI, EPI, false, false>(A, B, Out, ld, d.n, i0, j0, S.c1, S.c3, s0, s1, s2,
                                             red, &S.racc);
  else if (full)
    ns_gemm_rect_body<TI, EPI, false, true>(A, B, Out, ld, d.n, i0, j0, S.c1, S.c3, s0, s1, s2,
                                            red, &S.racc);
  else
    ns_gemm_rect_body<TI, EPI, true, false>(A, B, Out, ld, d.n, i0, j0, S.c1, S.c3, s0, s1, s2,
                                            red, &S.racc);
}

}  // namespace nolsm
