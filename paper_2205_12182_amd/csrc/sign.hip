// Batched Newton-Schulz sign iteration (paper, Eq. 6-7) on MFMA.
//
// Every iterate X_k is a polynomial in the symmetric M_k, so X_k, Y_k = X_k^2 and
// X_k Y_k are symmetric: each product is formed only on the upper-triangle
// ST x ST output tiles and mirrored into the lower triangle (this also keeps the
// iterates exactly symmetric).  One launch covers the tiles of every active
// submatrix of the batch (a grouped GEMM over submatrices of different n); a
// per-submatrix state word decides which submatrices still iterate.
//
// Per iteration:
//   ns_gemm<SQUARE>   Z = c1 I + c3 X X      and sum (X X - I)^2 for the residual
//   ns_check          residual, stop rule
//   ns_gemm<UPDATE>   X' = X Z               (Newton-Schulz: c1 = 3/2, c3 = -1/2)
//   ns_advance        X <- X', advance the spectral lower bound, next (c1, c3)
//
// The third-order step X' = 1/8 X (15 I - 10 X^2 + 3 X^4) uses the same two
// epilogues: since 15 - 10 y + 3 y^2 = 3 (y - 5/3)^2 + 20/3,
//   ns_gemm<SQUARE>   W = X X - 5/3 I        (residual of X X)
//   ns_check          residual, stop rule; the state now points at W
//   ns_gemm<SQUARE>   Z = 3/8 W W + 5/6 I
//   ns_shift          the state points at Z
//   ns_gemm<UPDATE>   X' = Z X  (= X Z: both are polynomials in the same M)
//   ns_advance
// The three buffers rotate so that the update writes W's buffer and the advance
// moves the state by two buffers, as for the Newton-Schulz step.
//
// Operands: both factors are read as column panels (A(m, k) = X(k, m) by
// symmetry), so every lane's MFMA fragment is a run of consecutive k.  The k
// order inside an LDS stage is permuted identically for A and B, which leaves the
// contraction unchanged and lets each lane read its whole stage slice as one
// 32-byte LDS access.
#include <type_traits>

#include "ns_gemm.h"
#include "ns_gemm_rect.h"

namespace nolsm {

// ------------------------------------------------------------------ per-submatrix control

struct PhaseArgs {
  int prec, t, iters, extra, use_lower, order;
  float tol;
  unsigned *live;     // the FP32 restart phase: restarting submatrices still iterating
};

// Coefficients (c1, c3) of the third-order step's two SQUARE epilogues.
constexpr float O3_W_C1 = -5.0f / 3.0f, O3_W_C3 = 1.0f;        // W = X^2 - 5/3 I
constexpr float O3_Z_C1 = 5.0f / 6.0f, O3_Z_C3 = 3.0f / 8.0f;  // Z = 3/8 W^2 + 5/6 I

// Spectrum-interval scaling of Newton-Schulz (Eq. 6 with a scaled argument): with
// every |eigenvalue| of X in [l, u], the step x <- p(a x), p(y) = y (3 - y^2) / 2,
// a^2 = 3 / (u^2 + u l + l^2), maps both ends of the interval to the same value
// p(a l) and keeps every eigenvalue up to sqrt(u^2 + u l + l^2) >= u positive
// (p(y) < 0 for y > sqrt 3).  The upper end is u = 1 + SCALE_MARGIN rather than 1:
// the low-precision iterates carry rounding errors that move eigenvalues near 1 by
// a few 1e-3 in FP16, and with u = 1 and a small l the margin sqrt(1 + l + l^2) - 1
// ~ l / 2 is smaller than that, which would send such eigenvalues to the wrong
// sign.  Once a <= 1 the plain step (a = 1) is used; its fixed points are exactly
// +-1.
constexpr double SCALE_MARGIN = 0.05;

__device__ __forceinline__ double ns_alpha(double l) {
  const double u = 1.0 + SCALE_MARGIN;
  const double a = sqrt(3.0 / (u * u + u * l + l * l));
  return a > 1.0 ? a : 1.0;
}

__device__ __forceinline__ double ns_p(double y) { return 0.5 * y * (3.0 - y * y); }

__device__ __forceinline__ void set_coeffs(SubState &s, int use_lower, int order) {
  if (order == 3) {
    s.c1 = O3_W_C1;
    s.c3 = O3_W_C3;
    return;
  }
  const double a = (use_lower && s.lower < 1.0) ? ns_alpha(s.lower) : 1.0;
  s.c1 = (float)(1.5 * a);
  s.c3 = (float)(-0.5 * a * a * a);
}

__global__ void ns_check_kernel(const SubDesc *__restrict__ desc, SubState *__restrict__ st,
                                int K, PhaseArgs p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  SubState &s = st[i];
  if (!s.active || s.prec != p.prec) return;
  // r = ||X^2 - I||_F bounds |1 - x^2| for every eigenvalue x of X, so r <= tol
  // certifies the whole spectrum (a mean-square measure would let a few slow
  // eigenvalues near the gap pass).
  const double sum = (double)s.racc * (1.0 / (double)(1ull << RESID_SHIFT));
  s.racc = 0ull;
  const float r = (float)sqrt(sum);
  (void)desc;
  s.resid = r;
  bool go;
  if (!(r < 1.0e3f)) {
    go = false;                                    // diverged or NaN
  } else if (p.tol > 0.0f) {
    if (s.extra_left < 0 && r <= p.tol) { s.extra_left = p.extra; s.converged = 1; }
    if (s.extra_left == 0) go = false;
    else {
      go = p.t < p.iters;
      if (s.extra_left > 0) --s.extra_left;
    }
  } else {
    go = p.t < p.iters;
  }
  if (!go) {
    s.active = 0;
    if (p.live) atomicSub(p.live, 1u);
  } else if (p.order == 3) {      // the next product squares W
    s.cur = (s.cur + 1) % 3;
    s.c1 = O3_Z_C1;
    s.c3 = O3_Z_C3;
  }
}

// Third-order step: the state moves from W to Z; the residual that the second
// SQUARE epilogue added (of W W, not X X) is dropped.
__global__ void ns_shift_kernel(SubState *__restrict__ st, int K, int prec) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  SubState &s = st[i];
  if (!s.active || s.prec != prec) return;
  s.cur = (s.cur + 1) % 3;
  s.racc = 0ull;
}

// rotate = 0 (the literal form, literal.hip): the buffers keep fixed roles.
__global__ void ns_advance_kernel(SubState *__restrict__ st, int K, int prec, int use_lower,
                                  int fallback, int order, int rotate, unsigned *live) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  SubState &s = st[i];
  if (!s.active || s.prec != prec) return;
  if (rotate) s.cur = (s.cur + 2) % 3;
  if (fallback) ++s.iters_fb; else ++s.iters_lo;
  if (s.extra_left == 0) {
    // a tolerance phase reached its tolerance and this was the last of its extra
    // iterations: stop now rather than after one more X^2, whose only use would be
    // the stop decision already taken (the residual on record stays the last one
    // measured, which met the tolerance)
    s.active = 0;
    if (live) atomicSub(live, 1u);
    return;
  }
  if (use_lower && s.lower < 1.0) {
    // new lower bound: the smaller image of the two interval ends
    const double l = s.lower, a = ns_alpha(l);
    const double pl = ns_p(a * l), pu = ns_p(a * (1.0 + SCALE_MARGIN));
    const double ln = pl < pu ? pl : pu;
    s.lower = ln > 1.0 ? 1.0 : ln;
  }
  set_coeffs(s, use_lower, order);    // for the next iteration's first SQUARE
}

// Start a phase: every healthy submatrix iterates; convert the current iterate
// if the phase changes precision (handled by convert_kernel on the host side).
__global__ void phase_start_kernel(SubState *__restrict__ st, int K, int use_lower,
                                   int only_fb, int order) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  SubState &s = st[i];
  if (s.status != 0) { s.active = 0; return; }
  if (only_fb && !s.fell_back) { s.active = 0; return; }
  s.active = 1;
  s.extra_left = -1;
  s.converged = 0;
  s.racc = 0ull;
  set_coeffs(s, use_lower, order);
}

__global__ void phase_end_kernel(SubState *__restrict__ st, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  st[i].active = 0;
}

// Convert the current iterate to precision `to` (one column per workgroup).
// Layouts: the iterate of a k-blocked submatrix (d.kb) is k-blocked in FP16 and BF16
// (the 256 x 128 tiles) and column major in FP32 (128 x 128 tiles).
template <typename TF, typename TT>
__device__ void convert_col(const TF *src, TT *dst, int ld, int c, bool kb_src, bool kb_dst) {
  for (int r = threadIdx.x; r < ld; r += blockDim.x) {
    const int64_t cm = (int64_t)c * ld + r;
    dst[kb_dst ? kb_index(r, c, ld) : cm] = from_f32<TT>(to_f32<TF>(src[kb_src ? kb_index(r, c, ld) : cm]));
  }
}

__global__ __launch_bounds__(256) void convert_kernel(const SubDesc *__restrict__ desc,
                                                      const SubState *__restrict__ st, char *ws,
                                                      int to) {
  const SubDesc d = desc[blockIdx.y];
  const SubState &s = st[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= d.npad || s.status != 0 || s.prec == to) return;
  const int q = s.cur, qn = (s.cur + 1) % 3;
  const bool ks = d.kb && s.prec != P_FP32, kd = d.kb && to != P_FP32;
#define CV(TF, TT) \
  convert_col<TF, TT>(buf_ptr<TF>(ws, d, q), buf_ptr<TT>(ws, d, qn), d.npad, c, ks, kd)
  if (s.prec == P_FP32 && to == P_FP16) CV(float, _Float16);
  else if (s.prec == P_FP32 && to == P_BF16) CV(float, __bf16);
  else if (s.prec == P_FP16 && to == P_FP32) CV(_Float16, float);
  else if (s.prec == P_FP16 && to == P_BF16) CV(_Float16, __bf16);
  else if (s.prec == P_BF16 && to == P_FP32) CV(__bf16, float);
  else if (s.prec == P_BF16 && to == P_FP16) CV(__bf16, _Float16);
#undef CV
}

__global__ void convert_commit_kernel(SubState *__restrict__ st, int K, int to) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  SubState &s = st[i];
  if (s.status != 0 || s.prec == to) return;
  s.cur = (s.cur + 1) % 3;
  s.prec = to;
}

// ------------------------------------------------------------------ scaling and X_0

// Gershgorin bound of M - mu I (symmetric: row sums = column sums), one wave per column.
__global__ __launch_bounds__(256) void gersh_kernel(const SubDesc *__restrict__ desc,
                                                    SubState *__restrict__ st, const char *ws,
                                                    double mu) {
  const SubDesc d = desc[blockIdx.y];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const float *M = reinterpret_cast<const float *>(ws + d.off_h);      // FP32 M
  double best = 0.0;
  for (int c = blockIdx.x * 64 + w * 16; c < blockIdx.x * 64 + w * 16 + 16; ++c) {
    if (c >= d.n) break;
    double s = 0.0;
    for (int r = lane; r < d.n; r += 64) {
      const double v = (double)M[(int64_t)c * d.npad + r];
      s += (r == c) ? fabs(v - mu) : fabs(v);
    }
    s = wave_sum(s);
    best = s > best ? s : best;
  }
  if (lane == 0 && best > 0.0)
    atomicMax(&st[blockIdx.y].scale_bits, (unsigned long long)__double_as_longlong(best));
}

// Pick b_k and l_k, reset the iteration state.  only_fb: restart fallback submatrices.
__global__ void scale_init_kernel(const SubDesc *__restrict__ desc, SubState *__restrict__ st,
                                  int K, const double *__restrict__ user_scale,
                                  const double *__restrict__ user_lower,
                                  const float *__restrict__ lower_log10, float lower_factor,
                                  int prec, int only_fb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  SubState &s = st[i];
  if (only_fb && !s.fell_back) return;
  double g = __longlong_as_double((long long)s.scale_bits);
  if (!(g > 0.0)) g = 1.0;
  s.scale = (user_scale && !only_fb) ? user_scale[i] : g;
  double l = 1.0;
  if (!only_fb) {
    if (user_lower) l = user_lower[i];
    else if (lower_log10) l = (double)lower_factor * pow(10.0, (double)lower_log10[i]);
  }
  s.lower = l < 1.0e-7 ? 1.0e-7 : (l > 1.0 ? 1.0 : l);
  s.prec = prec;
  s.cur = 0;
  s.racc = 0ull;
  s.active = (s.status == 0);
  s.extra_left = -1;
  s.converged = 0;
  if (!only_fb) { s.iters_lo = 0; s.iters_fb = 0; s.fell_back = 0; s.resid = 0.0f; }
}

// X_0 = (M - mu I) / b in the submatrix's precision; zero outside n x n.
// One wave per column, four consecutive rows per lane (16-byte reads of M); kb: the
// k-blocked layout (four consecutive rows stay adjacent).
template <typename TI>
__device__ __forceinline__ void cast_col4(const float *M, TI *X, int n, int ld, int c, double mu,
                                          double inv_b, bool kb = false) {
  typedef TI v4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  for (int q = lane; q < ld / 4; q += 64) {
    const int r = 4 * q;
    const float4 m = *reinterpret_cast<const float4 *>(M + (int64_t)c * ld + r);
    const float mv[4] = {m.x, m.y, m.z, m.w};
    v4 o;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double v = 0.0;
      if (r + e < n && c < n) v = ((double)mv[e] - (r + e == c ? mu : 0.0)) * inv_b;
      o[e] = from_f64<TI>(v);
    }
    *reinterpret_cast<v4 *>(X + (kb ? kb_index(r, c, ld) : (int64_t)c * ld + r)) = o;
  }
}

constexpr int CAST_COLS = 8;            // columns per workgroup (two per wave)

__global__ __launch_bounds__(256) void cast_kernel(const SubDesc *__restrict__ desc,
                                                   const SubState *__restrict__ st, char *ws,
                                                   double mu) {
  const SubDesc d = desc[blockIdx.y];
  const SubState &s = st[blockIdx.y];
  if (s.status != 0) return;
  const float *M = reinterpret_cast<const float *>(ws + d.off_h);      // FP32 M
  const double inv_b = 1.0 / s.scale;
  for (int c = blockIdx.x * CAST_COLS + (threadIdx.x >> 6); c < (blockIdx.x + 1) * CAST_COLS;
       c += 4) {
    if (c >= d.npad) break;
    if (s.prec == P_FP32) cast_col4<float>(M, buf_ptr<float>(ws, d, 0), d.n, d.npad, c, mu, inv_b);
    else if (s.prec == P_FP16)
      cast_col4<_Float16>(M, buf_ptr<_Float16>(ws, d, 0), d.n, d.npad, c, mu, inv_b, d.kb != 0);
    else cast_col4<__bf16>(M, buf_ptr<__bf16>(ws, d, 0), d.n, d.npad, c, mu, inv_b, d.kb != 0);
  }
}

// Fallback selection: not converged in a tolerance phase and residual above tol
// (or non-finite) -> restart from X_0 in FP32 with the Gershgorin scale.
// The selected submatrices are counted in *cnt and in *live (both cleared by
// clear_count_kernel); the restart phase takes each one off *live as it stops.
__global__ void fb_select_kernel(SubState *__restrict__ st, int K, float tol,
                                 unsigned *__restrict__ cnt, unsigned *__restrict__ live) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  SubState &s = st[i];
  s.active = 0;
  if (s.status != 0) return;
  if (!s.converged && !(s.resid <= tol)) {
    s.fell_back = 1;
    atomicAdd(cnt, 1u);
    atomicAdd(live, 1u);
  }
}

__global__ void clear_count_kernel(unsigned *__restrict__ cnt, unsigned *__restrict__ live) {
  *cnt = 0u;
  *live = 0u;
}

// X_0 of the restarting submatrices (FP32, column-major): grid (npad / CAST_FB_COLS,
// K), a wave per column at a time as in cast_kernel; every workgroup returns at once
// when nothing restarts.
constexpr int CAST_FB_COLS = 32;

__global__ __launch_bounds__(256) void cast_fb_kernel(const SubDesc *__restrict__ desc,
                                                      const SubState *__restrict__ st, char *ws,
                                                      double mu, const unsigned *__restrict__ cnt) {
  if (*cnt == 0u) return;
  const SubDesc d = desc[blockIdx.y];
  const SubState &s = st[blockIdx.y];
  if (s.status != 0 || !s.fell_back) return;
  const float *M = reinterpret_cast<const float *>(ws + d.off_h);      // FP32 M
  const double inv_b = 1.0 / s.scale;
  for (int c = blockIdx.x * CAST_FB_COLS + (threadIdx.x >> 6);
       c < (blockIdx.x + 1) * CAST_FB_COLS && c < d.npad; c += 4)
    cast_col4<float>(M, buf_ptr<float>(ws, d, 0), d.n, d.npad, c, mu, inv_b);
}

__global__ void fb_finish_kernel(SubState *__restrict__ st, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  SubState &s = st[i];
  s.active = 0;
  if (s.status == 0 && s.fell_back && !s.converged) s.status = NOLSM_ENOCONV;
}

__global__ void final_status_kernel(SubState *__restrict__ st, int K, int check_conv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  SubState &s = st[i];
  s.active = 0;
  if (check_conv && s.status == 0 && !s.converged) s.status = NOLSM_ENOCONV;
}

__global__ void clear_scale_kernel(SubState *__restrict__ st, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  st[i].scale_bits = 0ull;
}

// ------------------------------------------------------------------ host side

static inline int nblk(int K) { return (K + 255) / 256; }

void launch_reset_status(SubState *st, int K, int keep_spd, hipStream_t s);
void launch_lit_transpose(const SubDesc *desc, const SubState *st, int K, int max_npad, char *ws,
                          int mode, int prec, const unsigned *cnt, hipStream_t s);
void launch_lit_gemm(int square, const Tile *tiles, int ntiles, const SubDesc *desc, SubState *st,
                     char *ws, int prec, unsigned long long *flop_units, hipStream_t s);
void launch_lit_finish(SubState *st, int K, hipStream_t s);

template <typename TI, int EPI>
static void launch_ns_gemm_t(const TileSet &ts, const SubDesc *desc, SubState *st, char *ws,
                             int prec, hipStream_t s) {
  if (ts.n[0] > 0)
    ns_gemm_kernel<TI, EPI, 2><<<ts.n[0], 256, 0, s>>>(ts.t[0], desc, st, ws, prec,
                                                       ts.flop_units);
  if (std::is_same<TI, float>::value) {
    if (ts.n[2] > 0)
      ns_gemm_kernel<TI, EPI, 2><<<ts.n[2], 256, 0, s>>>(ts.t[2], desc, st, ws, prec,
                                                         ts.flop_units);
  } else if (ts.n[1] > 0) {
    ns_gemm_rect_kernel<typename std::conditional<std::is_same<TI, float>::value, _Float16,
                                                  TI>::type,
                        EPI><<<ts.n[1], 256, 0, s>>>(ts.t[1], desc, st, ws, prec, ts.flop_units);
  }
}

template <typename TI>
static void launch_ns_gemm(int epi, const TileSet &ts, const SubDesc *desc, SubState *st,
                           char *ws, int prec, hipStream_t s) {
  if (epi == EPI_SQUARE) launch_ns_gemm_t<TI, EPI_SQUARE>(ts, desc, st, ws, prec, s);
  else launch_ns_gemm_t<TI, EPI_UPDATE>(ts, desc, st, ws, prec, s);
}

static void ns_gemm(int epi, int prec, const TileSet &ts, const SubDesc *desc, SubState *st,
                    char *ws, hipStream_t s) {
  if (prec == P_FP32) launch_ns_gemm<float>(epi, ts, desc, st, ws, prec, s);
  else if (prec == P_FP16) launch_ns_gemm<_Float16>(epi, ts, desc, st, ws, prec, s);
  else launch_ns_gemm<__bf16>(epi, ts, desc, st, ws, prec, s);
}

void launch_final_status(SubState *st, int K, int check_conv, hipStream_t s) {
  final_status_kernel<<<nblk(K), 256, 0, s>>>(st, K, check_conv);
}

// One phase of the iteration (host loop of launches; no host synchronisation).
// FP32 restart products: tile lists 0 and 2 through the gated kernel.
static void gated_gemm(int epi, const TileSet &ts, const SubDesc *desc, SubState *st, char *ws,
                       hipStream_t s) {
  for (int l : {0, 2}) {
    if (ts.n[l] == 0) continue;
    const int grid = ts.n[l] < FB_GRID ? ts.n[l] : FB_GRID;
    if (epi == EPI_SQUARE)
      ns_gemm_gated_kernel<EPI_SQUARE><<<grid, 256, 0, s>>>(ts.t[l], ts.n[l], desc, st, ws,
                                                            ts.fb_live, ts.flop_units);
    else
      ns_gemm_gated_kernel<EPI_UPDATE><<<grid, 256, 0, s>>>(ts.t[l], ts.n[l], desc, st, ws,
                                                            ts.fb_live, ts.flop_units);
  }
}

static void timed_gemm(int epi, int prec, const TileSet &ts, const SubDesc *desc,
                       SubState *st, char *ws, EventLog *log, double flop, int fallback,
                       bool literal, hipStream_t s) {
  (void)flop;
  if (literal) {        // every tile of every submatrix (tile list 3), no gating
    const int e = (log && !fallback) ? log->begin(T_GEMM, s) : -1;
    launch_lit_gemm(epi == EPI_SQUARE, ts.t[3], ts.n[3], desc, st, ws, prec, ts.flop_units, s);
    if (e >= 0) {
      log->end(e, s);
      ++log->n_gemm;
    }
    return;
  }
  if (fallback) {
    gated_gemm(epi, ts, desc, st, ws, s);
    return;
  }
  const int e = log ? log->begin(T_GEMM, s) : -1;
  ns_gemm(epi, prec, ts, desc, st, ws, s);
  if (log && log->on) {
    log->end(e, s);
    ++log->n_gemm;
  }
}

void launch_phase(const SubDesc *desc, SubState *st, int K, int max_npad, const TileSet &ts,
                  char *ws, const nolsm_phase &ph, int use_lower, int fallback, EventLog *log,
                  double flop, bool literal, hipStream_t s) {
  PhaseArgs p;
  p.prec = ph.prec;
  p.iters = ph.iters;
  p.extra = ph.extra;
  p.tol = ph.tol;
  p.use_lower = use_lower;
  p.order = ph.order == 3 ? 3 : 2;
  p.live = fallback ? ts.fb_live : nullptr;
  const int last = (ph.tol > 0.0f) ? ph.iters : ph.iters - 1;
  for (int t = 0; t <= last; ++t) {
    p.t = t;
    timed_gemm(EPI_SQUARE, ph.prec, ts, desc, st, ws, log, flop, fallback, literal, s);
    ns_check_kernel<<<nblk(K), 256, 0, s>>>(desc, st, K, p);
    if (p.order == 3) {
      timed_gemm(EPI_SQUARE, ph.prec, ts, desc, st, ws, log, flop, fallback, literal, s);
      ns_shift_kernel<<<nblk(K), 256, 0, s>>>(st, K, ph.prec);
    }
    timed_gemm(EPI_UPDATE, ph.prec, ts, desc, st, ws, log, flop, fallback, literal, s);
    // the literal form keeps X^T beside X; transposed before the advance, which may
    // end a submatrix's iteration
    if (literal) launch_lit_transpose(desc, st, K, max_npad, ws, 1, ph.prec, nullptr, s);
    ns_advance_kernel<<<nblk(K), 256, 0, s>>>(st, K, ph.prec, use_lower, fallback, p.order,
                                              literal ? 0 : 1, p.live);
  }
  phase_end_kernel<<<nblk(K), 256, 0, s>>>(st, K);
}

// flop: executed MFMA flops of one GEMM launch over every tile of the plan.
// have_scale: the Gershgorin bounds for this mu are already in the state (written with
// the descriptors of the learned schedule), so the pass over M_k is skipped.
// literal: the literal form (literal.hip; one precision for every phase, order 2).
void launch_sign(const SubDesc *desc, SubState *st, int K, int max_npad, const TileSet &ts,
                 char *ws, double mu, const nolsm_schedule &sch, bool have_scale,
                 EventLog *log, double flop, bool literal, hipStream_t s) {
  launch_reset_status(st, K, 1, s);
  if (!have_scale) {
    clear_scale_kernel<<<nblk(K), 256, 0, s>>>(st, K);
    gersh_kernel<<<dim3(max_npad / 64, K), 256, 0, s>>>(desc, st, ws, mu);
  }
  scale_init_kernel<<<nblk(K), 256, 0, s>>>(desc, st, K, sch.scale, sch.lower, sch.lower_log10,
                                            sch.lower_factor, sch.phase[0].prec, 0);
  cast_kernel<<<dim3((max_npad + CAST_COLS - 1) / CAST_COLS, K), 256, 0, s>>>(desc, st, ws, mu);
  if (literal) launch_lit_transpose(desc, st, K, max_npad, ws, 0, 0, nullptr, s);
  for (int q = 0; q < sch.nphase; ++q) {
    const nolsm_phase &ph = sch.phase[q];
    if (q > 0 && ph.prec != sch.phase[q - 1].prec) {
      convert_kernel<<<dim3(max_npad, K), 256, 0, s>>>(desc, st, ws, ph.prec);
      convert_commit_kernel<<<nblk(K), 256, 0, s>>>(st, K, ph.prec);
    }
    const int scaled = (sch.lower != nullptr || sch.lower_log10 != nullptr) ? 1 : 0;
    phase_start_kernel<<<nblk(K), 256, 0, s>>>(st, K, scaled, 0, ph.order == 3 ? 3 : 2);
    launch_phase(desc, st, K, max_npad, ts, ws, ph, scaled, 0, log, flop, literal, s);
  }

  if (sch.fallback_iters > 0) {
    clear_count_kernel<<<1, 1, 0, s>>>(ts.fb_count, ts.fb_live);
    fb_select_kernel<<<nblk(K), 256, 0, s>>>(st, K, sch.fallback_tol, ts.fb_count, ts.fb_live);
    scale_init_kernel<<<nblk(K), 256, 0, s>>>(desc, st, K, nullptr, nullptr, nullptr, 0.0f,
                                              P_FP32, 1);
    cast_fb_kernel<<<dim3((max_npad + CAST_FB_COLS - 1) / CAST_FB_COLS, K), 256, 0, s>>>(
        desc, st, ws, mu, ts.fb_count);
    if (literal) launch_lit_transpose(desc, st, K, max_npad, ws, 2, 0, ts.fb_count, s);
    nolsm_phase fb;
    fb.prec = P_FP32;
    fb.iters = sch.fallback_iters;
    fb.tol = 1.0e-3f;
    fb.extra = 2;
    fb.order = 2;
    phase_start_kernel<<<nblk(K), 256, 0, s>>>(st, K, 0, 1, 2);
    launch_phase(desc, st, K, max_npad, ts, ws, fb, 0, 1, nullptr, 0.0, literal, s);
    fb_finish_kernel<<<nblk(K), 256, 0, s>>>(st, K);
  }
  if (literal) launch_lit_finish(st, K, s);      // the panel kernels read X^T
}

}  // namespace nolsm
