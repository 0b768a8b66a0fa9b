// Per-submatrix descriptors of A_k = M_k - mu I for the learned schedule.
//
// A is symmetric, so column statistics are row statistics.  Per column: the
// diagonal d = A_cc, the off-diagonal absolute sum R_c and the squared norm; per
// submatrix: Gershgorin bound b = max_c (|d| + R_c) and edges min (d - R),
// max (d + R), Tr A, ||A||_F^2 and diagonal moments.  The fixed thread-to-column
// assignment and combine order make the result reproducible.
#include <cfloat>

#include "common.h"

namespace nolsm {

struct ColAcc {
  double bmax, lo, hi, sd, sd2, sabsd, mind, sR, maxR, neg, f2;
};

__device__ __forceinline__ void acc_init(ColAcc &a) {
  a.bmax = 0.0; a.lo = DBL_MAX; a.hi = -DBL_MAX; a.sd = 0.0; a.sd2 = 0.0; a.sabsd = 0.0;
  a.mind = DBL_MAX; a.sR = 0.0; a.maxR = 0.0; a.neg = 0.0; a.f2 = 0.0;
}

__device__ __forceinline__ void acc_merge(ColAcc &a, const ColAcc &b) {
  a.bmax = fmax(a.bmax, b.bmax); a.lo = fmin(a.lo, b.lo); a.hi = fmax(a.hi, b.hi);
  a.sd += b.sd; a.sd2 += b.sd2; a.sabsd += b.sabsd; a.mind = fmin(a.mind, b.mind);
  a.sR += b.sR; a.maxR = fmax(a.maxR, b.maxR); a.neg += b.neg; a.f2 += b.f2;
}

// Pass 1: grid (npad / 64, K); workgroup x covers columns 64 x .. 64 x + 63, wave w
// columns 64 x + 16 w .. + 15, lanes stride down a column four rows at a time.  The
// workgroup's partial (waves combined in order) goes to the submatrix's set-up
// scratch (free once M is formed).
__global__ __launch_bounds__(256) void features_part_kernel(const SubDesc *__restrict__ desc,
                                                            char *ws, double mu) {
  const SubDesc d = desc[blockIdx.y];
  if ((int)blockIdx.x * 64 >= d.npad) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const float *M = reinterpret_cast<const float *>(ws + d.off_h);      // FP32 M
  ColAcc *part = reinterpret_cast<ColAcc *>(ws + d.off_diag);
  __shared__ ColAcc wp[4];
  ColAcc a;
  acc_init(a);
  const int cb = blockIdx.x * 64 + w * 16;
  for (int c = cb; c < cb + 16 && c < d.n; ++c) {
    double R = 0.0, f2 = 0.0, diag = 0.0;
    // four consecutive rows per lane (16-byte reads; npad is a multiple of 64)
    const float *col = M + (int64_t)c * d.npad;
#pragma unroll 2
    for (int r4 = 4 * lane; r4 < d.n; r4 += 256) {
      const float4 m4 = *reinterpret_cast<const float4 *>(col + r4);
      const float mv[4] = {m4.x, m4.y, m4.z, m4.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r4 + e;
        if (r >= d.n) break;
        double v = (double)mv[e];
        if (r == c) { v -= mu; diag = v; } else R += fabs(v);
        f2 += v * v;
      }
    }
    R = wave_sum(R);
    f2 = wave_sum(f2);
    diag = wave_sum(diag);                     // only one lane holds it
    a.bmax = fmax(a.bmax, fabs(diag) + R);
    a.lo = fmin(a.lo, diag - R);
    a.hi = fmax(a.hi, diag + R);
    a.sd += diag; a.sd2 += diag * diag; a.sabsd += fabs(diag);
    a.mind = fmin(a.mind, fabs(diag));
    a.sR += R; a.maxR = fmax(a.maxR, R);
    a.neg += diag < 0.0 ? 1.0 : 0.0;
    a.f2 += f2;
  }
  if (lane == 0) wp[w] = a;
  __syncthreads();
  if (threadIdx.x != 0) return;
  ColAcc t = wp[0];
  acc_merge(t, wp[1]);
  acc_merge(t, wp[2]);
  acc_merge(t, wp[3]);
  part[blockIdx.x] = t;
}

// Pass 2: one thread per submatrix combines the partials in column order.  The
// Gershgorin bound b = max_c sum_r |A_rc| also goes to the state as the scale of
// the sign iteration (the same quantity the sign call would otherwise compute).
__global__ __launch_bounds__(256) void features_final_kernel(const SubDesc *__restrict__ desc,
                                                             SubState *__restrict__ st,
                                                             const char *ws, int K,
                                                             float *__restrict__ feat) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const SubDesc d = desc[k];
  float *f = feat + (int64_t)k * NOLSM_NFEAT;
  const ColAcc *part = reinterpret_cast<const ColAcc *>(ws + d.off_diag);
  ColAcc t;
  acc_init(t);
  for (int x = 0; x < d.npad / 64; ++x) acc_merge(t, part[x]);
  const bool bad = st[k].status != 0 || d.n == 0;
  const double n = d.n > 0 ? (double)d.n : 1.0;
  const double b = t.bmax > 0.0 ? t.bmax : 1.0;
  const double rms = sqrt(t.f2 / n);
  const double mean = t.sd / n;
  const double var = fmax(t.sd2 / n - mean * mean, 0.0);
  float v[NOLSM_NFEAT] = {
      (float)log(n), (float)(d.nmem / 100.0), (float)(d.m / 32.0), (float)log(b),
      (float)(t.lo / b), (float)(t.hi / b), (float)(mean / b), (float)(rms / b),
      (float)(sqrt(var) / b), (float)(t.mind / b), (float)(t.sR / n / b), (float)(t.maxR / b),
      (float)(t.neg / n), (float)(t.sabsd / n / b), (float)(rms > 0.0 ? t.mind / rms : 0.0),
      1.0f};
  for (int i = 0; i < NOLSM_NFEAT; ++i) f[i] = bad ? 0.0f : v[i];
  st[k].scale_bits = t.bmax > 0.0 ? (unsigned long long)__double_as_longlong(t.bmax) : 0ull;
}

void launch_features(const SubDesc *desc, SubState *st, int K, int max_npad, char *ws,
                     double mu, float *feat, hipStream_t s) {
  features_part_kernel<<<dim3(max_npad / 64, K), 256, 0, s>>>(desc, ws, mu);
  features_final_kernel<<<(K + 255) / 256, 256, 0, s>>>(desc, st, ws, K, feat);
}

}  // namespace nolsm
