// Submatrix method, step 1 (paper, Sec. II; Eq. 8 for the non-orthogonal pair):
// gather the dense principal submatrices T_k(H0), T_k(S) of every planned molecule.
//
// One workgroup per (submatrix, member block column b).  It locates every block
// (J_a, J_b) of the submatrix in block column J_b by binary search, then streams
// the column-major block column into the dense column-major submatrix: each
// output column is a contiguous run of n doubles, so writes are coalesced, and
// each stored block is read contiguously.  The padding rows/columns (n..npad) are
// written as well: zero for H, the identity for S.  Of T_k(S) only the lower
// triangle (with the diagonal) is written: the factorisation reads nothing else,
// and the upper triangle is cleared before the inverse.
//
// SPLIT_H: T_k(H0) goes straight into the split FP16 operand of the set-up products
// (row j = column j by symmetry, npad hi parts then npad lo parts, x = hi + 2^-11 lo)
// instead of the FP64 H buffer.
#include "common.h"

namespace nolsm {

constexpr int GATHER_MAXMEM = 1024;     // members per submatrix held in LDS
constexpr int GATHER_MAXN = 8192;       // submatrix dimension held in the LDS row map

template <bool SPLIT_H>
__global__ __launch_bounds__(256) void gather_kernel(
    const SubDesc *__restrict__ desc, const int32_t *__restrict__ mem_mol,
    const int32_t *__restrict__ mem_loc, const int32_t *__restrict__ blk_dim,
    const int64_t *__restrict__ colptr, const int32_t *__restrict__ rowblk,
    const int64_t *__restrict__ valoff, const double *__restrict__ H_val,
    const double *__restrict__ S_val, char *__restrict__ ws) {
  const SubDesc d = desc[blockIdx.y];
  const int b = blockIdx.x;
  if (b > d.nmem) return;                       // b == nmem: padding columns
  __shared__ int64_t s_t[GATHER_MAXMEM];        // value offset of block (J_a, J_b) or -1
  __shared__ int32_t s_loc[GATHER_MAXMEM + 1];
  __shared__ int32_t s_dim[GATHER_MAXMEM];
  __shared__ uint16_t s_rowmem[GATHER_MAXN];    // row -> member
  double *Hk = reinterpret_cast<double *>(ws + d.off_h);
  double *Sk = reinterpret_cast<double *>(ws + d.off_s);
  const int n = d.n, ld = d.npad;
  _Float16 *Hs = reinterpret_cast<_Float16 *>(ws + d.off_lo) + 2 * (int64_t)ld * ld;   // buffer 1

  if (b == d.nmem) {                            // columns n..npad: zero / identity
    for (int c = n; c < ld; ++c)
      for (int r = threadIdx.x; r < ld; r += blockDim.x) {
        if (SPLIT_H) {
          Hs[(int64_t)c * 2 * ld + r] = (_Float16)0.0f;
          Hs[(int64_t)c * 2 * ld + ld + r] = (_Float16)0.0f;
        } else {
          Hk[(int64_t)c * ld + r] = 0.0;
        }
        Sk[(int64_t)c * ld + r] = (r == c) ? 1.0 : 0.0;
      }
    return;
  }

  const int Jb = mem_mol[d.mem_off + b];
  const int locb = mem_loc[d.mem_off + b];
  const int dJ = blk_dim[Jb];
  const int64_t c0 = colptr[Jb], c1 = colptr[Jb + 1];
  for (int a = threadIdx.x; a < d.nmem; a += blockDim.x) {
    const int Ja = mem_mol[d.mem_off + a];
    int64_t lo = c0, hi = c1;                   // first row >= Ja
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (rowblk[mid] < Ja) lo = mid + 1; else hi = mid;
    }
    s_t[a] = (lo < c1 && rowblk[lo] == Ja) ? valoff[lo] : -1;     // block values or absent
    s_loc[a] = mem_loc[d.mem_off + a];
    s_dim[a] = blk_dim[Ja];
  }
  __syncthreads();
  for (int a = 0; a < d.nmem; ++a)
    for (int r = threadIdx.x; r < s_dim[a]; r += blockDim.x) s_rowmem[s_loc[a] + r] = (uint16_t)a;
  __syncthreads();

  // column by column (32-bit index arithmetic, no per-element division); rows of
  // one member are contiguous in both the stored block and the output column
  for (int c = 0; c < dJ; ++c) {
    double *hcol = Hk + (int64_t)(locb + c) * ld;
    _Float16 *hrow = Hs + (int64_t)(locb + c) * 2 * ld;
    double *scol = Sk + (int64_t)(locb + c) * ld;
    const int col = locb + c;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
      double h = 0.0, sv = 0.0;
      if (i < n) {
        const int a = s_rowmem[i];
        const int64_t v0 = s_t[a];
        if (v0 >= 0) {
          const int64_t src = v0 + (i - s_loc[a]) + c * s_dim[a];
          h = H_val[src];
          if (i >= col) sv = S_val[src];
        }
      }
      if (SPLIT_H) {
        const _Float16 hi = (_Float16)h;                 // one rounding from FP64
        hrow[i] = hi;
        hrow[ld + i] = (_Float16)((h - (double)hi) * 2048.0);
      } else {
        hcol[i] = h;
      }
      if (i >= col) scol[i] = sv;               // the factorisation reads the lower triangle
    }
  }
}

void launch_gather(const SubDesc *desc, int K, int maxmem, const int32_t *mem_mol,
                   const int32_t *mem_loc, const nolsm_pattern *pat, const double *H_val,
                   const double *S_val, bool split_h, char *ws, hipStream_t stream) {
  dim3 grid(maxmem + 1, K);
  if (split_h)
    gather_kernel<true><<<grid, 256, 0, stream>>>(desc, mem_mol, mem_loc, pat->blk_dim,
                                                  pat->colptr, pat->rowblk, pat->valoff, H_val,
                                                  S_val, ws);
  else
    gather_kernel<false><<<grid, 256, 0, stream>>>(desc, mem_mol, mem_loc, pat->blk_dim,
                                                   pat->colptr, pat->rowblk, pat->valoff, H_val,
                                                   S_val, ws);
}

}  // namespace nolsm
