// Symmetric-product GEMM of the sign iteration (paper, Eq. 6): one launch covers
// the upper-triangle output tiles of every active submatrix of a batch.
//
// Workgroup: 256 threads = 4 waves in a 2 x 2 grid; each wave owns BMB x BMB
// blocks of 32 x 32 (v_mfma_f32_32x32x16_f16/bf16 or v_mfma_f32_32x32x2_f32), so
// the workgroup tile is (64 BMB)^2: 128 x 128 (BMB = 2) or 256 x 256 (BMB = 4).
//
// Both factors are read as column panels (A(m, k) = X(k, m) by symmetry): in
// every stage, row r of a panel is 64 contiguous bytes (32 FP16 or 16 FP32 k
// values, four 16-byte chunks).  Stages travel from memory straight into LDS
// (buffer loads with the LDS destination) through a ring of four slots, three
// stages ahead of the MFMAs; each slot is its own LDS array so that the
// compiler's wait-count tracking sees which slot a fragment read depends on,
// and the waits before each barrier are partial (only the stage about to be
// consumed).  Within a row the chunks are stored XOR-permuted by
// (r ^ (r >> 2)) & 3, which makes the 16-byte fragment reads free of bank
// conflicts without padding (measured with the hardware conflict counter: this
// permutation reads as fast as linear addresses, while ((r >> 1) ^ (r >> 3)) & 3
// costs 20% and 80-byte padded rows 60% extra LDS cycles).  Lane half h of an MFMA fragment takes chunks
// 2 h and 2 h + 1 of its row; the k order inside a stage is therefore permuted
// identically for A and B, which leaves the contraction unchanged.
//
// Tiles on the ragged edge (n padded to 64, tiles of 128/256) skip the 32 x 32
// blocks that lie entirely in the padding.
#pragma once
#include "common.h"

namespace nolsm {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f16x __attribute__((ext_vector_type(16)));
typedef float f4x __attribute__((ext_vector_type(4)));

// SQUARE: Z = c1 I + c3 X X (+ residual); UPDATE: X' = X Z; PLAIN_SYM: the plain
// product of a symmetric result (upper tiles, mirrored); PLAIN_FULL: the plain
// product, every tile, nothing mirrored; FULL_SQUARE: SQUARE's epilogue on every
// tile of a general (non-symmetric) product, nothing mirrored, the residual summed
// over every element once.
enum { EPI_SQUARE = 0, EPI_UPDATE = 1, EPI_PLAIN_SYM = 2, EPI_PLAIN_FULL = 3,
       EPI_FULL_SQUARE = 4 };

constexpr int NSLOT = 4;           // LDS ring slots (stages in flight: NSLOT - 1)
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

// One ring slot: the stage's A rows, then its B rows, 4 uint4 per row.
template <int BMB> __host__ __device__ constexpr int slot_u4() { return 2 * 64 * BMB * 4; }

template <typename TI>
__device__ __forceinline__ TI *buf_ptr(char *ws, const SubDesc &d, int q) {
  return reinterpret_cast<TI *>(ws + d.off_lo + (int64_t)q * 4 * d.npad * d.npad);
}

__device__ __forceinline__ int chunk_swz(int r) { return (r ^ (r >> 2)) & 3; }

// s_waitcnt immediate: wait until at most `vm` vector-memory operations are
// outstanding and every LDS operation has completed (expcnt left alone).
__host__ __device__ constexpr int wait_vm_lgkm0(int vm) {
  return (vm & 0xF) | ((vm >> 4) << 14) | (0x7 << 4);
}

#define NS_LDS_PTR(p) ((__attribute__((address_space(3))) void *)(p))

// C(m, c) = sum_{k < kend} A[m ld + k] B[c ld + k] for the tile at (i0, j0), i.e.
// C = A^T B for column-major A, B with leading dimension ld (kend: a multiple of
// the stage depth, at most ld).  TAG only separates instantiations made from
// different kernels (the host compilation pass rejects a second kernel that
// instantiates the same specialisation of this body).
template <typename TI, int EPI, int BMB, bool PARTIAL, int TAG = 0>
__device__ __forceinline__ void ns_gemm_body(const TI *__restrict__ A, const TI *__restrict__ B,
                                             TI *__restrict__ Out, int ld, int kend, int n, int i0,
                                             int j0,
                                             float c1, float c3, uint4 *s0, uint4 *s1, uint4 *s2,
                                             uint4 *s3, float *red, unsigned long long *racc) {
  constexpr int TILE = 64 * BMB;
  constexpr int LPS = TILE / 64;                 // loads per wave per operand per stage
  constexpr int BOFF = TILE * 4;                 // B rows start here within a slot (uint4)
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (w >> 1) * 32 * BMB, wn = (w & 1) * 32 * BMB;
  const int h = lane >> 5, l32 = lane & 31;
  const int nk = kend / KStage<TI>::KS;

  // blocks of this wave that hold rows/columns < ld
  int nvr = BMB, nvc = BMB;
  if (PARTIAL) {
    nvr = (ld - i0 - wm) / 32;
    nvc = (ld - j0 - wn) / 32;
    nvr = nvr < 0 ? 0 : (nvr > BMB ? BMB : nvr);
    nvc = nvc < 0 ? 0 : (nvc > BMB ? BMB : nvc);
  }

  // Panel loads go through buffer resources whose size is the npad x npad matrix:
  // rows past npad (ragged edge tiles) are out of range and read as zero.  Stages
  // past the last one are issued (every wave issues the same number of loads, so
  // the partial waits count right) against zero-size resources: nothing is read
  // and their slots are never consumed.
  const int nrec = ld * ld * (int)sizeof(TI);
  const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(A), (short)0, nrec, BUFFER_RSRC_WORD3);
  const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(B), (short)0, nrec, BUFFER_RSRC_WORD3);
  const __amdgpu_buffer_rsrc_t rA0 = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(A), (short)0, 0, BUFFER_RSRC_WORD3);
  const __amdgpu_buffer_rsrc_t rB0 = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TI *>(B), (short)0, 0, BUFFER_RSRC_WORD3);

  // A wave's load q fills rows 16 (4 q + w) .. + 15 of a panel: lane L writes the
  // 16 bytes at LDS offset 16 L of that 1 KiB block, i.e. row 16 (4 q + w) + L / 4,
  // slot L % 4, and so fetches chunk (L % 4) ^ chunk_swz(row) of the row.
  unsigned voA[LPS], voB[LPS];
#pragma unroll
  for (int q = 0; q < LPS; ++q) {
    const int row = 16 * (4 * q + w) + (lane >> 2);
    const unsigned ch = (unsigned)((lane & 3) ^ chunk_swz(row));
    voA[q] = (unsigned)((i0 + row) * ld) * (unsigned)sizeof(TI) + 16u * ch;
    voB[q] = (unsigned)((j0 + row) * ld) * (unsigned)sizeof(TI) + 16u * ch;
  }
  // Fragment reads: lane (h, l32) takes chunks 2 h and 2 h + 1 of rows
  // wm + 32 b + l32 (A) and wn + 32 b + l32 (B); the chunk permutation of those
  // rows depends on l32 only.
  const int z = chunk_swz(l32);
  const int fa0 = (wm + l32) * 4 + ((2 * h) ^ z), fa1 = (wm + l32) * 4 + ((2 * h + 1) ^ z);
  const int fb0 = BOFF + (wn + l32) * 4 + ((2 * h) ^ z),
            fb1 = BOFF + (wn + l32) * 4 + ((2 * h + 1) ^ z);

  f16x acc[BMB][BMB];
#pragma unroll
  for (int bm = 0; bm < BMB; ++bm)
#pragma unroll
    for (int bn = 0; bn < BMB; ++bn)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[bm][bn][q] = 0.0f;

  struct Frag { uint4 a[BMB][2], b[BMB][2]; };
  auto issue = [&](uint4 *slot, int kt) {
    const bool live = kt < nk;
    const __amdgpu_buffer_rsrc_t ra = live ? rA : rA0, rb = live ? rB : rB0;
    const int so = live ? 64 * kt : 0;
#pragma unroll
    for (int q = 0; q < LPS; ++q) {
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, NS_LDS_PTR(slot + (4 * q + w) * 64), 16,
                                               voA[q], so, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, NS_LDS_PTR(slot + BOFF + (4 * q + w) * 64),
                                               16, voB[q], so, 0, 0);
    }
  };
  auto read = [&](const uint4 *slot, Frag &f) {
#pragma unroll
    for (int b = 0; b < BMB; ++b) {
      f.a[b][0] = slot[fa0 + 128 * b];
      f.a[b][1] = slot[fa1 + 128 * b];
      f.b[b][0] = slot[fb0 + 128 * b];
      f.b[b][1] = slot[fb1 + 128 * b];
    }
  };
  // Stage kt is in registers (f).  Wait for stage kt + 1 to land (stages kt + 2
  // and kt + 3 may stay in flight) and for this wave's reads of stage kt; after
  // the barrier every wave is done with slot kt % NSLOT, which takes stage
  // kt + NSLOT.  Stage kt + 1 is read into g while the MFMAs consume f.
  // Instruction order inside a step (scheduling groups): the MFMAs are split into
  // NVM equal groups; inside each group half the MFMAs, then NDS / NVM fragment
  // reads and one LDS-destination load, then the other half.  The loads are
  // spread evenly, so a load that waits for space in the address unit's queue
  // delays few MFMAs; nothing moves across step boundaries.
  constexpr int NDS = 4 * BMB, NVM = 2 * LPS, NMF = BMB * BMB * Mfma<TI>::STEPS;
  constexpr int MPG = NMF / NVM;
  static_assert(NDS % NVM == 0 && NMF % NVM == 0 && MPG >= 2, "step interleave");
  auto step = [&](const uint4 *next, uint4 *refill, int kt, Frag &f, Frag &g) {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0((NSLOT - 2) * 2 * LPS));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    issue(refill, kt + NSLOT);
    read(next, g);
#pragma unroll
    for (int s = 0; s < Mfma<TI>::STEPS; ++s)
#pragma unroll
      for (int bm = 0; bm < BMB; ++bm)
#pragma unroll
        for (int bn = 0; bn < BMB; ++bn)
          if (!PARTIAL || (bm < nvr && bn < nvc))
            acc[bm][bn] = Mfma<TI>::op(f.a[bm], f.b[bn], s, acc[bm][bn]);
    if (!PARTIAL) {
#pragma unroll
      for (int j = 0; j < NVM; ++j) {
        __builtin_amdgcn_sched_group_barrier(0x008, MPG / 2, 0);          // MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, NDS / NVM, 0);        // LDS read
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);                // memory load
        __builtin_amdgcn_sched_group_barrier(0x008, MPG - MPG / 2, 0);    // MFMA
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  };

  Frag f, g;
  issue(s0, 0);
  issue(s1, 1);
  issue(s2, 2);
  issue(s3, 3);
  __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0((NSLOT - 1) * 2 * LPS));
  __builtin_amdgcn_s_barrier();
  read(s0, f);
  int kt = 0;
  for (; kt + NSLOT <= nk; kt += NSLOT) {
    step(s1, s0, kt, f, g);
    step(s2, s1, kt + 1, g, f);
    step(s3, s2, kt + 2, f, g);
    step(s0, s3, kt + 3, g, f);
  }
  const int rem = nk - kt;
  if (rem > 0) step(s1, s0, kt, f, g);
  if (rem > 1) step(s2, s1, kt + 1, g, f);
  if (rem > 2) step(s3, s2, kt + 2, f, g);
  // drain the trailing (empty) loads before the slots are reused for staging
  __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));
  __builtin_amdgcn_s_barrier();

  // Epilogue.  Element (r, c) of block (bm, bn), register q:
  //   r = wm + 32 bm + 8 (q >> 2) + 4 h + (q & 3),  c = wn + 32 bn + l32.
  // SQUARE turns X^2 into Z = c1 I + c3 X^2 (the residual is taken from X^2), so
  // UPDATE is the plain product X' = X Z.  Only elements with r <= c (global) are
  // kept, and each is stored to (r, c) and (c, r), so the result is exactly
  // symmetric.  The (c, r) stores go straight from registers (the 32 lanes of a
  // register hold 32 consecutive rows of column r of the output); the (r, c)
  // stores are staged in LDS, column major, and leave as 16-byte chunks.  The
  // staging tile is split by columns into four quarters, one per ring slot;
  // within a column the 16-byte chunk k sits at k ^ (column & 15).
  constexpr int CH = 16 / (int)sizeof(TI);                 // elements per 16-byte chunk
  constexpr int QC = TILE / 4;                              // columns per quarter
  static_assert(QC * TILE * (int)sizeof(TI) <= slot_u4<BMB>() * 16, "staging quarter");
  static_assert(TILE / CH >= 16, "chunk permutation needs 16 chunks per column");
  auto quarter = [&](int qi) -> TI * {
    return reinterpret_cast<TI *>(qi == 0 ? s0 : qi == 1 ? s1 : qi == 2 ? s2 : s3);
  };
  constexpr bool MIRROR = EPI != EPI_PLAIN_FULL && EPI != EPI_FULL_SQUARE;
  const bool diag_tile = MIRROR && (i0 == j0);
  // keep the row stride in a vector register so that the per-row store offsets
  // are formed with vector arithmetic instead of occupying scalar registers
  int ldv = ld;
  asm volatile("" : "+v"(ldv));
  float rs = 0.0f;     // diagonal tiles: weighted sum; other tiles: plain sum (weight 2 later)
#pragma unroll
  for (int bm = 0; bm < BMB; ++bm)
#pragma unroll
    for (int bn = 0; bn < BMB; ++bn) {
      if (PARTIAL && (bm >= nvr || bn >= nvc)) continue;
      const int c = wn + 32 * bn + l32, gc = j0 + c;
      TI *sq = quarter(c / QC) + (c % QC) * TILE;
      const int cz = c & 15;
      TI *mir = Out + (int64_t)(i0 + wm + 32 * bm + 4 * h) * ldv + gc;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int r0 = wm + 32 * bm + 8 * g + 4 * h;
        TI o[4];
        if (EPI == EPI_FULL_SQUARE) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int gr = i0 + r0 + e;
            const bool diag = gr == gc;
            float v = acc[bm][bn][4 * g + e];
            if (gr < n && gc < n) {
              const float df = v - (diag ? 1.0f : 0.0f);
              rs += df * df;
            }
            o[e] = from_f32<TI>(c3 * v + (diag && gc < n ? c1 : 0.0f));
          }
        } else if (!diag_tile) {          // every element has r < c (global)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            float v = acc[bm][bn][4 * g + e];
            if (EPI == EPI_SQUARE) {
              rs += v * v;
              v = c3 * v;
            }
            o[e] = from_f32<TI>(v);
            if (MIRROR) mir[(int64_t)(8 * g + e) * ldv] = o[e];
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
        typedef TI v4 __attribute__((ext_vector_type(4)));
        v4 ov;
#pragma unroll
        for (int e = 0; e < 4; ++e) ov[e] = o[e];
        *reinterpret_cast<v4 *>(sq + (((r0 / CH) ^ cz) * CH) + (r0 % CH)) = ov;
      }
    }
  __syncthreads();
  constexpr int CPC = TILE / CH;                             // chunks per column
  for (int idx = tid; idx < TILE * CPC; idx += 256) {
    const int c = idx / CPC, k = idx % CPC, row = k * CH;
    const int gc = j0 + c, gr0 = i0 + row;
    if (PARTIAL && (gc >= ld || gr0 >= ld)) continue;
    if (MIRROR && gr0 > gc) continue;
    const TI *src = quarter(c / QC) + (c % QC) * TILE + ((k ^ (c & 15)) * CH);
    TI *dst = Out + (int64_t)gc * ld + gr0;
    if (!MIRROR || gr0 + CH - 1 <= gc) {
      *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(src);
    } else {
      for (int e = 0; e < CH && gr0 + e <= gc; ++e) dst[e] = src[e];
    }
  }
  if (EPI == EPI_SQUARE) {
    // off-diagonal tiles count each element twice (it stands for (r, c) and (c, r));
    // their padding rows and columns are zero and contribute nothing
    const float tot = block_sum256(diag_tile ? rs : 2.0f * rs, red);
    if (tid == 0) atomicAdd(racc, resid_fixed(tot));
  }
  if (EPI == EPI_FULL_SQUARE) {
    const float tot = block_sum256(rs, red);
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
    atomicAdd(flop_units, (unsigned long long)((rows / 16) * (cols / 16) * (ld / 64)));
  }
  // the ring slots (separate arrays, see above); the epilogue reuses them as the
  // four column quarters of its staging tile
  __shared__ uint4 s0[slot_u4<BMB>()], s1[slot_u4<BMB>()], s2[slot_u4<BMB>()],
      s3[slot_u4<BMB>()];
  __shared__ float red[4];
  if (i0 + TILE <= ld && j0 + TILE <= ld)
    ns_gemm_body<TI, EPI, BMB, false>(A, B, Out, ld, ld, d.n, i0, j0, S.c1, S.c3, s0, s1, s2, s3,
                                      red, &S.racc);
  else
    ns_gemm_body<TI, EPI, BMB, true>(A, B, Out, ld, ld, d.n, i0, j0, S.c1, S.c3, s0, s1, s2, s3, red,
                                     &S.racc);
}

// FP32 products of the restart phase.  Usually no submatrix restarts, so the
// launches are gated: a small grid (at most FB_GRID workgroups, two per CU) walks
// the tile list in rounds and every workgroup returns at once when no restarting
// submatrix is still iterating (the count the stop decisions decrement).  Within a round, consecutive tiles go to one XCD as above.
constexpr int FB_GRID = 512;

template <int EPI>
__global__ __launch_bounds__(256) void ns_gemm_gated_kernel(
    const Tile *__restrict__ tiles, int ntiles, const SubDesc *__restrict__ desc,
    SubState *__restrict__ st, char *ws, const unsigned *__restrict__ gate,
    unsigned long long *__restrict__ flop_units) {
  if (*gate == 0u) return;
  __shared__ uint4 s0[slot_u4<2>()], s1[slot_u4<2>()], s2[slot_u4<2>()], s3[slot_u4<2>()];
  __shared__ float red[4];
  for (int base = 0; base < ntiles; base += gridDim.x) {
    const int cnt = ntiles - base < (int)gridDim.x ? ntiles - base : (int)gridDim.x;
    if ((int)blockIdx.x >= cnt) break;
    const Tile t = tiles[base + xcd_remap(blockIdx.x, cnt)];
    SubState &S = st[t.sub];
    if (!S.active || S.prec != P_FP32) continue;
    const SubDesc d = desc[t.sub];
    const int ld = d.npad;
    const int cur = S.cur;
    const float *A = buf_ptr<float>(ws, d, cur);
    const float *B = (EPI == EPI_SQUARE) ? A : buf_ptr<float>(ws, d, (cur + 1) % 3);
    float *Out = buf_ptr<float>(ws, d, (cur + (EPI == EPI_SQUARE ? 1 : 2)) % 3);
    const int i0 = t.ti * 128, j0 = t.tj * 128;
    if (threadIdx.x == 0) {
      const int rows = (ld - i0 < 128 ? ld - i0 : 128), cols = (ld - j0 < 128 ? ld - j0 : 128);
      atomicAdd(flop_units, (unsigned long long)((rows / 16) * (cols / 16) * (ld / 64)));
    }
    if (i0 + 128 <= ld && j0 + 128 <= ld)
      ns_gemm_body<float, EPI, 2, false, 1>(A, B, Out, ld, ld, d.n, i0, j0, S.c1, S.c3, s0, s1,
                                            s2, s3, red, &S.racc);
    else
      ns_gemm_body<float, EPI, 2, true, 1>(A, B, Out, ld, ld, d.n, i0, j0, S.c1, S.c3, s0, s1,
                                           s2, s3, red, &S.racc);
    __syncthreads();             // the ring slots are refilled by the next tile
  }
}

// Set-up products in FP32 (128 x 128 tiles), on the three FP32 buffers of the
// iteration arena: buffer 0 = L^-T, buffer 1 = H, buffer 2 = U.
//   PLAIN_FULL: U = H L^-T, every tile; L^-T(k, c) = 0 for k > c, so the
//               contraction stops at the tile's last column.
//   PLAIN_SYM:  M = L^-1 U (symmetric), upper tiles mirrored, written in FP32 over
//               the FP64 H buffer (H is no longer needed); L^-1(r, k) = 0 for k > r,
//               so the contraction stops at the tile's last row.
template <int EPI>
__global__ __launch_bounds__(256) void setup_gemm_kernel(const Tile *__restrict__ tiles,
                                                         const SubDesc *__restrict__ desc,
                                                         const SubState *__restrict__ st,
                                                         char *ws) {
  constexpr int TILE = 128;
  const Tile t = tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (st[t.sub].status != 0) return;
  const SubDesc d = desc[t.sub];
  const int ld = d.npad;
  float *Lt = buf_ptr<float>(ws, d, 0), *H = buf_ptr<float>(ws, d, 1), *U = buf_ptr<float>(ws, d, 2);
  float *M = reinterpret_cast<float *>(ws + d.off_h);      // FP32 M over the FP64 H buffer
  const int i0 = t.ti * TILE, j0 = t.tj * TILE;
  const float *A = EPI == EPI_PLAIN_FULL ? H : Lt;
  const float *B = EPI == EPI_PLAIN_FULL ? Lt : U;
  float *Out = EPI == EPI_PLAIN_FULL ? U : M;
  const int kl = (EPI == EPI_PLAIN_FULL ? j0 : i0) + TILE;
  const int kend = kl < ld ? kl : ld;
  __shared__ uint4 s0[slot_u4<2>()], s1[slot_u4<2>()], s2[slot_u4<2>()], s3[slot_u4<2>()];
  __shared__ float red[4];
  if (i0 + TILE <= ld && j0 + TILE <= ld)
    ns_gemm_body<float, EPI, 2, false>(A, B, Out, ld, kend, d.n, i0, j0, 0.0f, 0.0f, s0, s1, s2,
                                       s3, red, nullptr);
  else
    ns_gemm_body<float, EPI, 2, true>(A, B, Out, ld, kend, d.n, i0, j0, 0.0f, 0.0f, s0, s1, s2, s3,
                                      red, nullptr);
}

}  // namespace nolsm
