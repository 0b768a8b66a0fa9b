// Symmetric-product GEMM of the sign iteration (paper, Eq. 6): one launch covers
// the upper-triangle output tiles of every active submatrix of a batch.
//
// Workgroup: 256 threads = 4 waves in a 2 x 2 grid; each wave owns BMB x BMB
// blocks of 32 x 32 (v_mfma_f32_32x32x16_f16/bf16 or v_mfma_f32_32x32x2_f32), so
// the workgroup tile is (64 BMB)^2: 128 x 128 (BMB = 2) or 256 x 256 (BMB = 4).
//
// Both factors are read as column panels (A(m, k) = X(k, m) by symmetry): in
// every LDS stage, row r of a panel is 64 contiguous bytes (32 FP16 or 16 FP32 k
// values), staged through registers into a double-buffered LDS ring with 80-byte
// rows (16 bytes of padding keep the fragment reads free of bank conflicts).
// Lane half h of an MFMA fragment takes the 32 bytes at offset 32 h of its row;
// the k order inside a stage is therefore permuted identically for A and B,
// which leaves the contraction unchanged.
//
// Tiles on the ragged edge (n padded to 64, tiles of 128/256) skip the 32 x 32
// blocks that lie entirely in the padding.
#pragma once
#include "common.h"

namespace nolsm {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f16x __attribute__((ext_vector_type(16)));

enum { EPI_SQUARE = 0, EPI_UPDATE = 1 };

constexpr int LROW16 = 5;          // LDS row: 80 bytes = 5 x uint4 (64 data + 16 pad)
// Word 3 of a raw (stride 0) buffer resource on CDNA: 32-bit data format, no
// swizzle; offsets at or beyond num_records return zero.
constexpr int BUFFER_RSRC_WORD3 = 0x00020000;

template <typename TI> struct KStage;
template <> struct KStage<_Float16> { static constexpr int KS = 32; };
template <> struct KStage<__bf16> { static constexpr int KS = 32; };
template <> struct KStage<float> { static constexpr int KS = 16; };

template <typename TI> struct Mfma;
template <> struct Mfma<_Float16> {
  static constexpr int STEPS = 2;            // MFMAs per 64-byte stage slice
  __device__ static __forceinline__ f16x op(const uint4 (&a)[2], const uint4 (&b)[2], int s,
                                            f16x c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8, a[s]),
                                                  __builtin_bit_cast(h8, b[s]), c, 0, 0, 0);
  }
};
template <> struct Mfma<__bf16> {
  static constexpr int STEPS = 2;
  __device__ static __forceinline__ f16x op(const uint4 (&a)[2], const uint4 (&b)[2], int s,
                                            f16x c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(b8, a[s]),
                                                   __builtin_bit_cast(b8, b[s]), c, 0, 0, 0);
  }
};
__device__ __forceinline__ unsigned u4_word(const uint4 &v, int i) {
  return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}
template <> struct Mfma<float> {
  static constexpr int STEPS = 8;
  __device__ static __forceinline__ f16x op(const uint4 (&a)[2], const uint4 (&b)[2], int s,
                                            f16x c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(
        __builtin_bit_cast(float, u4_word(a[s >> 2], s & 3)),
        __builtin_bit_cast(float, u4_word(b[s >> 2], s & 3)), c, 0, 0, 0);
  }
};

// LDS for the epilogue's column-major staging tile: TILE columns of TILE + 8
// elements, in one round or (if that exceeds EPI_LDS_BYTES) two rounds of half
// the columns.
constexpr int EPI_LDS_BYTES = 135168;
template <typename TI, int TILE>
__host__ __device__ constexpr int smem_epi_u4() {
  return ((int)sizeof(TI) * TILE * (TILE + 8) > EPI_LDS_BYTES ? (int)sizeof(TI) * TILE * (TILE + 8) / 2
                                                               : (int)sizeof(TI) * TILE * (TILE + 8)) /
         16;
}

template <typename TI>
__device__ __forceinline__ TI *buf_ptr(char *ws, const SubDesc &d, int q) {
  return reinterpret_cast<TI *>(ws + d.off_lo + (int64_t)q * 4 * d.npad * d.npad);
}

template <typename TI, int EPI, int BMB, bool PARTIAL>
__device__ __forceinline__ void ns_gemm_body(const TI *__restrict__ A, const TI *__restrict__ B,
                                             TI *__restrict__ Out, int ld, int n, int i0, int j0,
                                             float c1, float c3, uint4 *sA, uint4 *sB,
                                             float *red, unsigned long long *racc) {
  constexpr int TILE = 64 * BMB;
  constexpr int SU4 = TILE * LROW16;             // uint4 per operand per LDS stage
  constexpr int U4T = TILE * 4 / 256;            // uint4 loaded per thread per operand
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * 32 * BMB, wn = (w & 1) * 32 * BMB;
  const int h = lane >> 5, l32 = lane & 31;
  const int nk = ld / KStage<TI>::KS;

  // blocks of this wave that hold rows/columns < ld
  int nvr = BMB, nvc = BMB;
  if (PARTIAL) {
    nvr = (ld - i0 - wm) / 32;
    nvc = (ld - j0 - wn) / 32;
    nvr = nvr < 0 ? 0 : (nvr > BMB ? BMB : nvr);
    nvc = nvc < 0 ? 0 : (nvc > BMB ? BMB : nvc);
  }

  // Panel loads go through buffer resources whose size is the npad x npad matrix:
  // rows past npad (ragged edge tiles) are out of range and read as zero.
  const int nrec = ld * ld * (int)sizeof(TI);
  const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(A), (short)0, nrec, BUFFER_RSRC_WORD3);
  const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(B), (short)0, nrec, BUFFER_RSRC_WORD3);
  unsigned voA[U4T], voB[U4T];
  int lofs[U4T];
#pragma unroll
  for (int q = 0; q < U4T; ++q) {
    const int row = (tid >> 2) + 64 * q, ch = tid & 3;
    voA[q] = (unsigned)((i0 + row) * ld) * (unsigned)sizeof(TI) + 16u * ch;
    voB[q] = (unsigned)((j0 + row) * ld) * (unsigned)sizeof(TI) + 16u * ch;
    lofs[q] = row * LROW16 + ch;
  }
  uint4 ra[U4T], rb[U4T];
#pragma unroll
  for (int q = 0; q < U4T; ++q) {
    ra[q] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rA, voA[q], 0, 0));
    rb[q] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rB, voB[q], 0, 0));
  }
#pragma unroll
  for (int q = 0; q < U4T; ++q) {
    sA[lofs[q]] = ra[q];
    sB[lofs[q]] = rb[q];
  }
  __syncthreads();

  f16x acc[BMB][BMB];
#pragma unroll
  for (int bm = 0; bm < BMB; ++bm)
#pragma unroll
    for (int bn = 0; bn < BMB; ++bn)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[bm][bn][q] = 0.0f;

  for (int kt = 0; kt < nk; ++kt) {
    const int cur = (kt & 1) * SU4, nxt = SU4 - cur;
    if (kt + 1 < nk) {
      const unsigned o = 64u * (unsigned)(kt + 1);
#pragma unroll
      for (int q = 0; q < U4T; ++q) {
        ra[q] = __builtin_bit_cast(uint4,
                                   __builtin_amdgcn_raw_buffer_load_b128(rA, voA[q] + o, 0, 0));
        rb[q] = __builtin_bit_cast(uint4,
                                   __builtin_amdgcn_raw_buffer_load_b128(rB, voB[q] + o, 0, 0));
      }
    }
    uint4 af[BMB][2], bf[BMB][2];
#pragma unroll
    for (int bm = 0; bm < BMB; ++bm) {
      const int r = (wm + bm * 32 + l32) * LROW16 + h * 2 + cur;
      af[bm][0] = sA[r];
      af[bm][1] = sA[r + 1];
    }
#pragma unroll
    for (int bn = 0; bn < BMB; ++bn) {
      const int r = (wn + bn * 32 + l32) * LROW16 + h * 2 + cur;
      bf[bn][0] = sB[r];
      bf[bn][1] = sB[r + 1];
    }
#pragma unroll
    for (int s = 0; s < Mfma<TI>::STEPS; ++s)
#pragma unroll
      for (int bm = 0; bm < BMB; ++bm)
#pragma unroll
        for (int bn = 0; bn < BMB; ++bn)
          if (!PARTIAL || (bm < nvr && bn < nvc))
            acc[bm][bn] = Mfma<TI>::op(af[bm], bf[bn], s, acc[bm][bn]);
    if (kt + 1 < nk) {
#pragma unroll
      for (int q = 0; q < U4T; ++q) {
        sA[nxt + lofs[q]] = ra[q];
        sB[nxt + lofs[q]] = rb[q];
      }
    }
    __syncthreads();
  }

  // Epilogue.  Element (r, c) of block (bm, bn), register q:
  //   r = wm + 32 bm + 8 (q >> 2) + 4 h + (q & 3),  c = wn + 32 bn + l32.
  // SQUARE turns X^2 into Z = c1 I + c3 X^2 (the residual is taken from X^2), so
  // UPDATE is the plain product X' = X Z.  Only elements with r <= c (global) are
  // kept, and each is stored to (r, c) and (c, r), so the result is exactly
  // symmetric.  The (c, r) stores go straight from registers (the 32 lanes of a
  // register hold 32 consecutive rows of column r of the output); the (r, c)
  // stores are staged in LDS, column major, and leave as 16-byte chunks.
  constexpr int CH = 16 / (int)sizeof(TI);                 // elements per 16-byte chunk
  constexpr int LSTR = TILE + 8;                            // LDS column stride (elements)
  constexpr int ROUNDS = ((int)sizeof(TI) * TILE * LSTR > EPI_LDS_BYTES) ? 2 : 1;
  constexpr int RCOLS = TILE / ROUNDS;
  TI *sT = reinterpret_cast<TI *>(sA);
  const bool diag_tile = (i0 == j0);
  // keep the row stride in a vector register so that the per-row store offsets
  // are formed with vector arithmetic instead of occupying scalar registers
  int ldv = ld;
  asm volatile("" : "+v"(ldv));
  float rs = 0.0f;     // diagonal tiles: weighted sum; other tiles: plain sum (weight 2 later)
#pragma unroll
  for (int rd = 0; rd < ROUNDS; ++rd) {
    if (ROUNDS == 1 || wn / RCOLS == rd) {
#pragma unroll
      for (int bm = 0; bm < BMB; ++bm)
#pragma unroll
        for (int bn = 0; bn < BMB; ++bn) {
          if (PARTIAL && (bm >= nvr || bn >= nvc)) continue;
          const int c = wn + 32 * bn + l32, gc = j0 + c;
          TI *mir = Out + (int64_t)(i0 + wm + 32 * bm + 4 * h) * ldv + gc;
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const int r0 = wm + 32 * bm + 8 * g + 4 * h;
            TI o[4];
            if (!diag_tile) {          // every element has r < c (global)
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                float v = acc[bm][bn][4 * g + e];
                if (EPI == EPI_SQUARE) {
                  rs += v * v;
                  v = c3 * v;
                }
                o[e] = from_f32<TI>(v);
                mir[(int64_t)(8 * g + e) * ldv] = o[e];
              }
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
                o[e] = from_f32<TI>(v);
                if (gr < gc) mir[(int64_t)(8 * g + e) * ldv] = o[e];
              }
            }
            TI *dst = sT + (c - rd * RCOLS) * LSTR + r0;
#pragma unroll
            for (int e = 0; e < 4; ++e) dst[e] = o[e];
          }
        }
    }
    __syncthreads();
    constexpr int CPC = TILE / CH;                           // chunks per column
    for (int idx = tid; idx < RCOLS * CPC; idx += 256) {
      const int cl = idx / CPC, row = (idx % CPC) * CH;
      const int gc = j0 + rd * RCOLS + cl, gr0 = i0 + row;
      if (PARTIAL && (gc >= ld || gr0 >= ld)) continue;
      const TI *src = sT + cl * LSTR + row;
      TI *dst = Out + (int64_t)gc * ld + gr0;
      if (gr0 + CH - 1 <= gc) {
        *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(src);
      } else if (gr0 <= gc) {
        for (int e = 0; e < CH && gr0 + e <= gc; ++e) dst[e] = src[e];
      }
    }
    if (ROUNDS > 1) __syncthreads();
  }
  if (EPI == EPI_SQUARE) {
    // off-diagonal tiles count each element twice (it stands for (r, c) and (c, r));
    // their padding rows and columns are zero and contribute nothing
    const float tot = block_sum256(diag_tile ? rs : 2.0f * rs, red);
    if (tid == 0) atomicAdd(racc, resid_fixed(tot));
  }
}

// SQUARE: Z = c1 I + c3 X X (+ residual of X X);  UPDATE: X' = X Z.
template <typename TI, int EPI, int BMB>
__global__ __launch_bounds__(256) void ns_gemm_kernel(const Tile *__restrict__ tiles,
                                                      const SubDesc *__restrict__ desc,
                                                      SubState *__restrict__ st, char *ws,
                                                      int prec,
                                                      unsigned long long *__restrict__ flop_units) {
  constexpr int TILE = 64 * BMB;
  const Tile t = tiles[xcd_remap(blockIdx.x, gridDim.x)];
  SubState &S = st[t.sub];
  if (!S.active || S.prec != prec) return;
  const SubDesc d = desc[t.sub];
  const int ld = d.npad;
  const int cur = S.cur;
  const TI *A = buf_ptr<TI>(ws, d, cur);
  const TI *B = (EPI == EPI_SQUARE) ? A : buf_ptr<TI>(ws, d, (cur + 1) % 3);
  TI *Out = buf_ptr<TI>(ws, d, (cur + (EPI == EPI_SQUARE ? 1 : 2)) % 3);
  const int i0 = t.ti * TILE, j0 = t.tj * TILE;
  if (threadIdx.x == 0) {
    const int rows = (ld - i0 < TILE ? ld - i0 : TILE), cols = (ld - j0 < TILE ? ld - j0 : TILE);
    atomicAdd(flop_units, (unsigned long long)((rows / 32) * (cols / 32) * (ld / 64)));
  }
  // one LDS union: the main loop's two double-buffered operand rings, then the
  // epilogue's staging tile
  constexpr int MAIN_U4 = 4 * TILE * LROW16;
  constexpr int EPI_U4 = smem_epi_u4<TI, TILE>();
  __shared__ uint4 smem[MAIN_U4 > EPI_U4 ? MAIN_U4 : EPI_U4];
  __shared__ float red[4];
  uint4 *sA = smem, *sB = smem + 2 * TILE * LROW16;
  if (i0 + TILE <= ld && j0 + TILE <= ld)
    ns_gemm_body<TI, EPI, BMB, false>(A, B, Out, ld, d.n, i0, j0, S.c1, S.c3, sA, sB, red,
                                      &S.racc);
  else
    ns_gemm_body<TI, EPI, BMB, true>(A, B, Out, ld, d.n, i0, j0, S.c1, S.c3, sA, sB, red,
                                     &S.racc);
}

}  // namespace nolsm
