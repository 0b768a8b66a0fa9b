// Set-up products M = L^-1 H L^-T on FP16 MFMAs with split operands.
//
// Each FP32-class operand x is stored as two FP16 numbers, x = hi + 2^-11 lo with
// hi = fp16(x) and lo = fp16(2^11 (x - hi)); the representation error is at most
// 2^-22 |x| (for |x| above the FP16 normal range floor, 2^-14; below it the error
// is absolute, under 2^-36).  A product of two such operands keeps three of the
// four partial products,
//   a b  ~  hi_a hi_b + 2^-11 (hi_a lo_b + lo_a hi_b),
// dropping 2^-22 lo_a lo_b, so every term of the contraction is within about
// 3 * 2^-22 |a| |b| of its exact value and the sums are FP32.  That is FP32-class
// accuracy (FP32 operands carry 2^-24) for three FP16 MFMA passes, which run
// about five times faster than one pass of FP32 MFMAs.
//
// Operand layout: a split matrix holds hi(X) in its first npad^2 FP16 values and
// lo(X) in the next npad^2, each k-blocked by rows: element k of row r at
// ((k / 32) npad + r) 32 + k % 32 (split_index), so that 32 k of 256 consecutive rows,
// one stage of a panel, are one contiguous block (as for the sign iterate, kb_index).  The contraction runs over
// three segments of k, the two correction products first:
//   segment 0: hi_A lo_B,  segment 1: lo_A hi_B,  then acc *= 2^-11,  segment 2: hi_A hi_B
// so the corrections are accumulated at the scale of hi and the final FP32 sum
// carries no extra rounding from the 2^-11 factor (a power of two).
//
// Tiles are 256 x 128 with four waves and two workgroups per CU, staged as in the
// sign-iteration kernel (direct-to-LDS loads two stages ahead from contiguous stage
// blocks, 64-byte rows with the chunk permutation).
//   SPLIT_FULL: U = H L^-T on every tile; the result is written split (rows of U'
//               are the columns of U), ready to be the B operand of the next product.
//               L^-T(k, c) = 0 for k > c, so the contraction stops at the tile's
//               last column.
//   SPLIT_SYM:  M = L^-1 U on the upper tiles, FP32, mirrored so that M is exactly
//               symmetric.  L^-1(r, k) = 0 for k > r, so the contraction stops at
//               the tile's last row.
#pragma once
#include "ns_gemm.h"
#include "ns_gemm_rect.h"

namespace nolsm {

enum { SPLIT_FULL = 0, SPLIT_SYM = 1 };
constexpr float SPLIT_LO_SCALE = 2048.0f;        // 2^11
constexpr float SPLIT_LO_UNSCALE = 1.0f / 2048.0f;

// Element k of row r of a split matrix's hi (lo: + npad^2) part.
__host__ __device__ __forceinline__ int64_t split_index(int r, int k, int np) {
  return ((int64_t)(k >> 5) * np + r) * 32 + (k & 31);
}

__device__ __forceinline__ void split_f16(float v, _Float16 &hi, _Float16 &lo) {
  hi = (_Float16)v;
  lo = (_Float16)((v - (float)hi) * SPLIT_LO_SCALE);
}
__device__ __forceinline__ void split_f16(double v, _Float16 &hi, _Float16 &lo) {
  hi = (_Float16)v;                               // one rounding from FP64
  lo = (_Float16)((v - (double)hi) * (double)SPLIT_LO_SCALE);
}

// C(m, c) = sum_k A(m, k) B(c, k) over k < kend for the tile at (i0, j0); A and B
// are split matrices (row stride 2 npad FP16).
template <int EPI, bool PARTIAL>
__device__ __forceinline__ void split_gemm_body(const _Float16 *__restrict__ A,
                                                const _Float16 *__restrict__ B, void *Out, int np,
                                                int kend, int i0, int j0, uint4 *s0, uint4 *s1,
                                                uint4 *s2) {
  typedef _Float16 TI;
  constexpr int BM = 4, BN = 2;
  constexpr int LA = RT_M / 64, LB = RT_N / 64;
  constexpr int LPS = LA + LB;
  constexpr int BOFF = RT_M * 4;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (w >> 1) * 32 * BM, wn = (w & 1) * 32 * BN;
  const int h = lane >> 5, l32 = lane & 31;
  const int nks = kend / KStage<TI>::KS;         // stages per segment
  const int nk = 3 * nks;
  const int lo_bytes = np * np * (int)sizeof(TI);   // byte offset of the lo part
  constexpr unsigned OOB = 0x80000000u;            // past the buffer: reads as zero

  int nvr = BM, nvc = BN;
  if (PARTIAL) {
    nvr = (np - i0 - wm) / 32;
    nvc = (np - j0 - wn) / 32;
    nvr = nvr < 0 ? 0 : (nvr > BM ? BM : nvr);
    nvc = nvc < 0 ? 0 : (nvc > BN ? BN : nvc);
  }

  // rows past npad (ragged edge tiles) read as zero; stages past the last one are
  // issued against zero-size resources so every wave issues the same loads
  const int nrec = 2 * np * np * (int)sizeof(TI);
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
    voA[q] = i0 + row < np ? (unsigned)(i0 + row) * 64u + 16u * ch : OOB;
  }
#pragma unroll
  for (int q = 0; q < LB; ++q) {
    const int row = 16 * (4 * q + w) + (lane >> 2);
    const unsigned ch = (unsigned)((lane & 3) ^ chunk_swz(row));
    voB[q] = j0 + row < np ? (unsigned)(j0 + row) * 64u + 16u * ch : OOB;
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
    const int seg = (kt >= nks) + (kt >= 2 * nks);
    const int kb = 64 * np * (kt - seg * nks);     // the stage's block
    const __amdgpu_buffer_rsrc_t ra = live ? rA : rA0, rb = live ? rB : rB0;
    const int soa = live ? kb + (seg == 1 ? lo_bytes : 0) : 0;
    const int sob = live ? kb + (seg == 0 ? lo_bytes : 0) : 0;
#pragma unroll
    for (int q = 0; q < LA; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, NS_LDS_PTR(slot + (4 * q + w) * 64), 16,
                                               voA[q], soa, 0, 0);
#pragma unroll
    for (int q = 0; q < LB; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, NS_LDS_PTR(slot + BOFF + (4 * q + w) * 64),
                                               16, voB[q], sob, 0, 0);
  };
  constexpr int NDS = 2 * (BM + BN), NMF = BM * BN * Mfma<TI>::STEPS;
  const int kscale = 2 * nks;
  auto step = [&](const uint4 *cur, uint4 *refill, int kt) {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(LPS));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    if (kt == kscale) {                 // corrections done: bring them to the scale of hi
#pragma unroll
      for (int bm = 0; bm < BM; ++bm)
#pragma unroll
        for (int bn = 0; bn < BN; ++bn)
#pragma unroll
          for (int q = 0; q < 16; ++q) acc[bm][bn][q] *= SPLIT_LO_UNSCALE;
    }
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
  __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));

  // Epilogue from registers.  Element (r, c) of block (bm, bn), register q:
  //   r = wm + 32 bm + 8 (q >> 2) + 4 h + (q & 3),  c = wn + 32 bn + l32.
  int ldv = np;
  asm volatile("" : "+v"(ldv));
  if (EPI == SPLIT_FULL) {
    // U(r, c) -> element r of row c of U': hi at split_index(c, r), lo np^2 after it
    TI *U = reinterpret_cast<TI *>(Out);
    const int64_t lo_off = (int64_t)ldv * ldv;
    typedef TI v4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < BN; ++bn) {
        if (PARTIAL && (bm >= nvr || bn >= nvc)) continue;
        const int gc = j0 + wn + 32 * bn + l32;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int r0 = wm + 32 * bm + 8 * g + 4 * h;
          TI *row = U + split_index(gc, i0 + r0, ldv);     // four consecutive k
          v4 hv, lv;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            TI a, b;
            split_f16(acc[bm][bn][4 * g + e], a, b);
            hv[e] = a;
            lv[e] = b;
          }
          *reinterpret_cast<v4 *>(row) = hv;
          *reinterpret_cast<v4 *>(row + lo_off) = lv;
        }
      }
  } else {
    // M(r, c), r <= c: to M[c np + r] and, for r < c, the mirror M[r np + c]
    float *M = reinterpret_cast<float *>(Out);
    const bool cross = (i0 < j0 + RT_N) && (j0 < i0 + RT_M);
    typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < BN; ++bn) {
        if (PARTIAL && (bm >= nvr || bn >= nvc)) continue;
        const int c = wn + 32 * bn + l32, gc = j0 + c;
        float *col = M + (int64_t)gc * ldv + i0;
        float *mir = M + (int64_t)(i0 + wm + 32 * bm + 4 * h) * ldv + gc;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int r0 = wm + 32 * bm + 8 * g + 4 * h;
          if (!cross) {
            f4 ov;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              ov[e] = acc[bm][bn][4 * g + e];
              mir[(int64_t)(8 * g + e) * ldv] = ov[e];
            }
            *reinterpret_cast<f4 *>(col + r0) = ov;
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int gr = i0 + r0 + e;
              const float v = acc[bm][bn][4 * g + e];
              if (gr <= gc) col[r0 + e] = v;
              if (gr < gc) mir[(int64_t)(8 * g + e) * ldv] = v;
            }
          }
        }
      }
  }
}

// Split FP16 operands in the iteration arena: buffer 0 = L^-1 (rows), buffer 1 = H
// (rows), buffer 2 = U' (rows = columns of U); M goes to the FP64 H buffer as FP32.
template <int EPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void split_gemm_kernel(const Tile *__restrict__ tiles, const SubDesc *__restrict__ desc,
                       const SubState *__restrict__ st, char *ws) {
  const Tile t = tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (st[t.sub].status != 0) return;
  const SubDesc d = desc[t.sub];
  const int np = d.npad;
  const _Float16 *Ls = buf_ptr<_Float16>(ws, d, 0), *Hs = buf_ptr<_Float16>(ws, d, 1);
  _Float16 *Us = buf_ptr<_Float16>(ws, d, 2);
  const int i0 = t.ti * RT_M, j0 = t.tj * RT_N;
  const _Float16 *A = EPI == SPLIT_FULL ? Hs : Ls;
  const _Float16 *B = EPI == SPLIT_FULL ? Ls : Us;
  void *Out = EPI == SPLIT_FULL ? (void *)Us : (void *)(ws + d.off_h);
  const int kl = EPI == SPLIT_FULL ? j0 + RT_N : i0 + RT_M;
  const int kend = kl < np ? kl : np;
  __shared__ uint4 s0[RT_SLOT_U4], s1[RT_SLOT_U4], s2[RT_SLOT_U4];
  if (i0 + RT_M <= np && j0 + RT_N <= np)
    split_gemm_body<EPI, false>(A, B, Out, np, kend, i0, j0, s0, s1, s2);
  else
    split_gemm_body<EPI, true>(A, B, Out, np, kend, i0, j0, s0, s1, s2);
}

}  // namespace nolsm
