// Submatrix method, step 1 (paper, Sec. II; Eq. 8 for the non-orthogonal pair):
// gather the dense principal submatrices T_k(H0), T_k(S) of every planned molecule.
//
// One workgroup per (submatrix, group of four member block columns b).  The member
// list goes to LDS once with a row -> member map and the members in ascending
// molecule order; for each b the stored blocks of block column J_b are read once,
// coalesced, and each is matched to its member by a binary search in LDS.  The workgroup then streams the column-major block column
// into the dense column-major submatrix, four consecutive rows per thread: each
// output column is a contiguous run, so writes are coalesced vector stores, and
// each stored block is read contiguously.  The padding rows/columns (n..npad) are
// written as well: zero for H, the identity for S.  Of T_k(S) only the lower
// triangle (with the diagonal) is written: the factorisation reads nothing else,
// and the upper triangle is cleared before the inverse.
//
// SPLIT_H: T_k(H0) goes straight into the split FP16 operand of the set-up products
// (row j = column j by symmetry, hi parts then lo parts, x = hi + 2^-11 lo, k-blocked
// as split_index says) instead of the FP64 H buffer.
#include "common.h"
#include "ns_gemm_split.h"

namespace nolsm {

constexpr int GATHER_MAXMEM = 1024;     // members per submatrix held in LDS
constexpr int GATHER_MAXN = 8192;       // submatrix dimension held in the LDS row map
constexpr int GATHER_GROUP = 4;         // member block columns per workgroup

template <bool SPLIT_H>
__global__ __launch_bounds__(256) void gather_kernel(
    const SubDesc *__restrict__ desc, const int32_t *__restrict__ mem_mol,
    const int32_t *__restrict__ mem_loc, const int32_t *__restrict__ blk_dim,
    const int32_t *__restrict__ mem_srt, const int64_t *__restrict__ colptr,
    const int32_t *__restrict__ rowblk,
    const int64_t *__restrict__ valoff, const double *__restrict__ H_val,
    const double *__restrict__ S_val, char *__restrict__ ws) {
  const SubDesc d = desc[blockIdx.y];
  const int nmem = d.nmem;
  const int b0 = blockIdx.x * GATHER_GROUP;     // member block columns b0 .. b0 + GROUP - 1
  if (b0 > nmem) return;                        // b == nmem stands for the padding columns
  const int b1 = b0 + GATHER_GROUP - 1 < nmem ? b0 + GATHER_GROUP - 1 : nmem;
  __shared__ int64_t s_t[GATHER_MAXMEM];        // value offset of block (J_a, J_b) or -1
  __shared__ int32_t s_loc[GATHER_MAXMEM + 1];  // first row of member a; s_loc[nmem] = n
  __shared__ int32_t s_mol[GATHER_MAXMEM];      // molecules in ascending order ...
  __shared__ int16_t s_pos[GATHER_MAXMEM];      // ... and their member indices
  __shared__ uint16_t s_rowmem[GATHER_MAXN];    // row -> member
  double *Hk = reinterpret_cast<double *>(ws + d.off_h);
  double *Sk = reinterpret_cast<double *>(ws + d.off_s);
  const int n = d.n, ld = d.npad;
  _Float16 *Hs = reinterpret_cast<_Float16 *>(ws + d.off_lo) + 2 * (int64_t)ld * ld;   // buffer 1

  if (b0 < nmem) {                              // the member list and row map, once
    for (int a = threadIdx.x; a < nmem; a += blockDim.x) {
      const int Ja = mem_mol[d.mem_off + a];
      const int loc = mem_loc[d.mem_off + a], dim = blk_dim[Ja];
      const int q = mem_srt[d.mem_off + a];        // a-th smallest molecule's member index
      s_mol[a] = mem_mol[d.mem_off + q];
      s_pos[a] = (int16_t)q;
      s_loc[a] = loc;
      for (int r = 0; r < dim; ++r) s_rowmem[loc + r] = (uint16_t)a;
    }
    if (threadIdx.x == 0) s_loc[nmem] = n;
  }

  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  for (int b = b0; b <= b1; ++b) {
    if (b == nmem) {                            // columns n..npad: zero / identity
      for (int c = n; c < ld; ++c)
        for (int r = threadIdx.x; r < ld; r += blockDim.x) {
          if (SPLIT_H) {
            Hs[split_index(c, r, ld)] = (_Float16)0.0f;
            Hs[split_index(c, r, ld) + (int64_t)ld * ld] = (_Float16)0.0f;
          } else {
            Hk[(int64_t)c * ld + r] = 0.0;
          }
          Sk[(int64_t)c * ld + r] = (r == c) ? 1.0 : 0.0;
        }
      break;
    }
    const int Jb = mem_mol[d.mem_off + b];
    const int locb = mem_loc[d.mem_off + b];
    const int dJ = blk_dim[Jb];
    const int64_t c0 = colptr[Jb], c1 = colptr[Jb + 1];
    __syncthreads();                             // the previous column set is done with s_t
    for (int a = threadIdx.x; a < nmem; a += blockDim.x) s_t[a] = -1;   // absent by default
    __syncthreads();
    for (int64_t e = c0 + threadIdx.x; e < c1; e += blockDim.x) {
      const int J = rowblk[e];
      int lo = 0, hi = nmem;                     // first member >= J
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_mol[mid] < J) lo = mid + 1; else hi = mid;
      }
      if (lo < nmem && s_mol[lo] == J) s_t[s_pos[lo]] = valoff[e];   // rows are distinct
    }
    __syncthreads();

    // column by column (32-bit index arithmetic, no per-element division); rows of
    // one member are contiguous in both the stored block and the output column.
    // ld is a multiple of 64, so every four-row group lies inside the column.
    for (int c = 0; c < dJ; ++c) {
      double *hcol = Hk + (int64_t)(locb + c) * ld;
      const int64_t hlo = (int64_t)ld * ld;              // lo part after the hi part
      double *scol = Sk + (int64_t)(locb + c) * ld;
      const int col = locb + c;
      for (int i0 = 4 * threadIdx.x; i0 < ld; i0 += 4 * blockDim.x) {
        double h[4], sv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = i0 + e;
          h[e] = 0.0;
          sv[e] = 0.0;
          if (i < n) {
            const int a = s_rowmem[i];
            const int64_t v0 = s_t[a];
            if (v0 >= 0) {
              const int64_t src = v0 + (i - s_loc[a]) + c * (s_loc[a + 1] - s_loc[a]);
              h[e] = H_val[src];
              if (i >= col) sv[e] = S_val[src];
            }
          }
        }
        if (SPLIT_H) {
          h4 hi, lo;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            hi[e] = (_Float16)h[e];                      // one rounding from FP64
            lo[e] = (_Float16)((h[e] - (double)hi[e]) * 2048.0);
          }
          _Float16 *hp = Hs + split_index(locb + c, i0, ld);   // row locb + c, k = i0 .. i0 + 3
          *reinterpret_cast<h4 *>(hp) = hi;
          *reinterpret_cast<h4 *>(hp + hlo) = lo;
        } else {
          *reinterpret_cast<double2 *>(hcol + i0) = make_double2(h[0], h[1]);
          *reinterpret_cast<double2 *>(hcol + i0 + 2) = make_double2(h[2], h[3]);
        }
        // the factorisation reads the lower triangle only
        if (i0 >= col) {
          *reinterpret_cast<double2 *>(scol + i0) = make_double2(sv[0], sv[1]);
          *reinterpret_cast<double2 *>(scol + i0 + 2) = make_double2(sv[2], sv[3]);
        } else if (i0 + 3 >= col) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (i0 + e >= col) scol[i0 + e] = sv[e];
        }
      }
    }
  }
}

void launch_gather(const SubDesc *desc, int K, int maxmem, const int32_t *mem_mol,
                   const int32_t *mem_loc, const int32_t *mem_srt, const nolsm_pattern *pat,
                   const double *H_val, const double *S_val, bool split_h, char *ws,
                   hipStream_t stream) {
  dim3 grid((maxmem + GATHER_GROUP) / GATHER_GROUP, K);   // members 0..maxmem (padding)
  if (split_h)
    gather_kernel<true><<<grid, 256, 0, stream>>>(desc, mem_mol, mem_loc, pat->blk_dim,
                                                  mem_srt, pat->colptr, pat->rowblk, pat->valoff, H_val,
                                                  S_val, ws);
  else
    gather_kernel<false><<<grid, 256, 0, stream>>>(desc, mem_mol, mem_loc, pat->blk_dim,
                                                   mem_srt, pat->colptr, pat->rowblk, pat->valoff, H_val,
                                                   S_val, ws);
}

}  // namespace nolsm
