// C ABI of the NOLSM library: planning, workspace layout and the entry points.
#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.h"

namespace nolsm {
void launch_gather(const SubDesc *desc, int K, int maxmem, const int32_t *mem_mol,
                   const int32_t *mem_loc, const int32_t *mem_srt, const nolsm_pattern *pat,
                   const double *H_val, const double *S_val, bool split_h, char *ws,
                   hipStream_t stream);
void launch_setup(const SubDesc *desc, SubState *st, int K, int max_npad, const TileSet &ts,
                  bool fp32_products, bool factor_fp32, bool literal, char *ws, hipStream_t s);
void launch_sign(const SubDesc *desc, SubState *st, int K, int max_npad, const TileSet &ts,
                 char *ws, double mu, const nolsm_schedule &sch, bool have_scale,
                 EventLog *log, double flop, bool literal, hipStream_t s);
void launch_density_columns(const SubDesc *desc, const SubState *st, int K, int max_npad,
                            int max_m, char *ws, int panel_steps, bool literal, hipStream_t s);
void launch_scatter(const SubDesc *desc, const SubState *st, int K, int maxmem,
                    const int32_t *mem_mol, const int32_t *mem_loc, const int32_t *mem_srt,
                    const nolsm_pattern *pat, double *D_val, const double *H_val,
                    const double *S_val, const char *ws, nolsm_stats *stats, hipStream_t s);
void launch_energy(const nolsm_pattern *pat, int nmol, const double *D_val, const double *H_val,
                   const double *S_val, double *col_traces, double *out2, hipStream_t s);
void launch_stats(const SubDesc *desc, const SubState *st, int K, nolsm_stats *out,
                  hipStream_t s);
void launch_trace_x(const SubDesc *desc, SubState *st, int K, const char *ws, hipStream_t s);
hipError_t energy_scratch_ptr(double **out);
void launch_final_status(SubState *st, int K, int check_conv, hipStream_t s);
void launch_features(const SubDesc *desc, SubState *st, int K, int max_npad, char *ws,
                     double mu, float *feat, hipStream_t s);
}  // namespace nolsm

using namespace nolsm;

struct nolsm_plan {
  int32_t K = 0;
  int32_t nmol = 0;
  int32_t maxmem = 0;
  int32_t max_npad = 0;
  std::vector<SubDesc> desc;
  std::vector<int32_t> mem_mol, mem_loc;
  std::vector<int32_t> mem_srt; // per submatrix: member indices by ascending molecule
  int32_t max_m = 0;            // most own columns of a submatrix
  std::vector<Tile> tiles;      // the tile lists of TileSet, back to back
  int32_t list_end[NTILELIST] = {};
  bool setup_fp32 = false;      // set-up products on FP32 MFMAs instead of split FP16
  bool factor_fp64 = false;     // factorisation and inverse tile products on FP64 MFMAs
  bool literal = false;         // the literal form of Eq. 8 (NOLSM_FORM_LITERAL)
  bool persist = false;         // M_k and L^-1 in the plan's own buffer (offsets off_h, off_s
                                // of desc[] are then relative to that buffer)
  size_t persist_bytes = 0;
  char *persist_buf = nullptr;  // persist buffer of the last upload
  // tables (bytes from the plan's table buffer)
  size_t off_desc = 0, off_mem_mol = 0, off_mem_loc = 0, off_mem_srt = 0, off_tiles = 0,
         off_state = 0;
  size_t tab_bytes = 0;
  // workspace (bytes from the workspace base)
  size_t off_counter = 0;       // unsigned long long: executed sign-GEMM work (FLOP_UNIT),
                                // then two unsigned: FP32 restarts, and of those the
                                // ones still iterating
  size_t bytes = 0;
  char *tab = nullptr;          // table buffer the tables were last uploaded to
  char *tab_ws = nullptr;       // workspace of the last upload (persist plans: the uploaded
                                // offsets depend on the workspace and persist pointers)
  char *ws = nullptr;
  bool bound = false;
  bool setup_done = false;      // M_k and L^-1 are current (set-up ran after the last gather)
  bool scale_ready = false;     // the Gershgorin bounds of M_k - scale_mu I are in the state
  double scale_mu = 0.0;        //   (written by nolsm_features after the last set-up)
  double gemm_flop = 0.0;       // executed MFMA flops of one sign GEMM launch (all tiles)
  EventLog log;
};

static thread_local std::string g_err;

static nolsm_status fail(nolsm_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static nolsm_status fail(nolsm_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

namespace nolsm {
nolsm_status set_error(nolsm_status code, const char *msg) { return fail(code, "%s", msg); }
}  // namespace nolsm

static nolsm_status hip_check(const char *where) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NOLSM_EHIP, "%s: %s", where, hipGetErrorString(e));
  return NOLSM_OK;
}

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

extern "C" {

const char *nolsm_last_error(void) { return g_err.c_str(); }

nolsm_status nolsm_plan_create(const nolsm_pattern *pat, const int32_t *mols, int32_t K,
                               nolsm_plan **out) {
  return nolsm_plan_create_ex(pat, mols, K, nullptr, out);
}

static nolsm_status plan_build(const nolsm_pattern *pat, const int32_t *grp_ptr,
                               const int32_t *grp_mols, int32_t K, const nolsm_plan_options *opt,
                               nolsm_plan **out);

nolsm_status nolsm_plan_create_ex(const nolsm_pattern *pat, const int32_t *mols, int32_t K,
                                  const nolsm_plan_options *opt, nolsm_plan **out) {
  if (!pat || !out || (K > 0 && !mols) || K < 0)
    return fail(NOLSM_EINVAL, "nolsm_plan_create: null argument or K < 0");
  std::vector<int32_t> ptr(K + 1);
  for (int i = 0; i <= K; ++i) ptr[i] = i;
  return plan_build(pat, ptr.data(), mols, K, opt, out);
}

nolsm_status nolsm_plan_create_groups(const nolsm_pattern *pat, const int32_t *grp_ptr,
                                      const int32_t *grp_mols, int32_t ngroups,
                                      const nolsm_plan_options *opt, nolsm_plan **out) {
  if (!pat || !out || !grp_ptr || ngroups < 0 || (ngroups > 0 && !grp_mols))
    return fail(NOLSM_EINVAL, "nolsm_plan_create_groups: null argument or ngroups < 0");
  if (grp_ptr[0] != 0)
    return fail(NOLSM_EINVAL, "nolsm_plan_create_groups: grp_ptr[0] must be 0");
  for (int g = 0; g < ngroups; ++g)
    if (grp_ptr[g + 1] <= grp_ptr[g])
      return fail(NOLSM_EINVAL, "nolsm_plan_create_groups: group %d is empty", g);
  return plan_build(pat, grp_ptr, grp_mols, ngroups, opt, out);
}

static nolsm_status plan_build(const nolsm_pattern *pat, const int32_t *grp_ptr,
                               const int32_t *grp_mols, int32_t K, const nolsm_plan_options *opt,
                               nolsm_plan **out) {
  int big_min = BIG_TILE_MIN_NPAD;
  bool setup_fp32 = false, persist = false, factor_fp64 = false, literal = false;
  if (opt) {
    for (int i = 0; i < 3; ++i)
      if (opt->reserved[i] != 0)
        return fail(NOLSM_EINVAL, "nolsm_plan_create_ex: reserved option field %d is not zero", i);
    if (opt->setup_products != 0 && opt->setup_products != 1)
      return fail(NOLSM_EINVAL, "nolsm_plan_create_ex: setup_products must be 0 or 1, got %d",
                  opt->setup_products);
    if (opt->persist != 0 && opt->persist != 1)
      return fail(NOLSM_EINVAL, "nolsm_plan_create_ex: persist must be 0 or 1, got %d",
                  opt->persist);
    if (opt->factor_tiles != 0 && opt->factor_tiles != 1)
      return fail(NOLSM_EINVAL, "nolsm_plan_create_ex: factor_tiles must be 0 or 1, got %d",
                  opt->factor_tiles);
    if (opt->form != NOLSM_FORM_SYM && opt->form != NOLSM_FORM_LITERAL)
      return fail(NOLSM_EINVAL, "nolsm_plan_create_ex: form must be 0 or 1, got %d", opt->form);
    if (opt->big_tile_min_npad >= 0) big_min = opt->big_tile_min_npad;
    setup_fp32 = opt->setup_products == 1;
    persist = opt->persist == 1;
    factor_fp64 = opt->factor_tiles == 1;
    literal = opt->form == NOLSM_FORM_LITERAL;
  }
  if (!pat->blk_dim || !pat->blk_off || !pat->colptr || !pat->rowblk || !pat->valoff)
    return fail(NOLSM_EINVAL, "nolsm_plan_create: pattern arrays must be set (host copies)");
  nolsm_plan *p = new (std::nothrow) nolsm_plan;
  if (!p) return fail(NOLSM_ENOMEM, "nolsm_plan_create: out of host memory");
  p->K = K;
  p->nmol = pat->nmol;
  p->setup_fp32 = setup_fp32;
  p->factor_fp64 = factor_fp64;
  p->literal = literal;
  p->persist = persist;
  p->desc.resize(K);
  size_t off = 0;
  std::vector<char> used(pat->nmol > 0 ? pat->nmol : 1, 0);
  std::vector<int32_t> grp, rows;
  auto bad = [&](nolsm_status code, const std::string &msg) {
    delete p;
    return fail(code, "%s", msg.c_str());
  };
  for (int i = 0; i < K; ++i) {
    // the group's molecules, ascending, each in range and in no other group
    grp.assign(grp_mols + grp_ptr[i], grp_mols + grp_ptr[i + 1]);
    std::sort(grp.begin(), grp.end());
    for (size_t a = 0; a < grp.size(); ++a) {
      const int k = grp[a];
      if (k < 0 || k >= pat->nmol)
        return bad(NOLSM_EINVAL, "nolsm_plan_create: molecule " + std::to_string(k) +
                                     " (submatrix " + std::to_string(i) + ") out of range");
      if (used[k])
        return bad(NOLSM_EINVAL, "nolsm_plan_create: molecule " + std::to_string(k) +
                                     " planned twice");
      used[k] = 1;
    }
    // rows: the union of the group's block columns (each ascending, with its diagonal)
    rows.clear();
    for (const int k : grp) {
      const int64_t c0 = pat->colptr[k], c1 = pat->colptr[k + 1];
      bool diag = false;
      for (int64_t t = c0; t < c1; ++t) {
        const int J = pat->rowblk[t];
        if (t > c0 && J <= pat->rowblk[t - 1])
          return bad(NOLSM_EINVAL, "nolsm_plan_create: rows of block column " +
                                       std::to_string(k) + " not ascending");
        diag |= J == k;
        rows.push_back(J);
      }
      if (!diag)
        return bad(NOLSM_EINVAL, "nolsm_plan_create: diagonal block (" + std::to_string(k) +
                                     ", " + std::to_string(k) + ") not stored");
    }
    std::sort(rows.begin(), rows.end());
    rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
    // member order: one molecule keeps the ascending rows; a combined group comes
    // first (ascending), then the other rows ascending, so that its own columns are
    // contiguous
    std::vector<int32_t> order;
    int own_mem = 0;
    if (grp.size() == 1) {
      order = rows;
      own_mem = (int)(std::lower_bound(order.begin(), order.end(), grp[0]) - order.begin());
    } else {
      order = grp;
      for (const int J : rows)
        if (!std::binary_search(grp.begin(), grp.end(), J)) order.push_back(J);
    }
    SubDesc &d = p->desc[i];
    std::memset(&d, 0, sizeof d);
    d.mol = grp[0];
    d.ngrp = (int32_t)grp.size();
    d.own_mem = own_mem;
    d.mem_off = (int32_t)p->mem_mol.size();
    d.nmem = (int32_t)order.size();
    int loc = 0;
    for (const int J : order) {
      p->mem_mol.push_back(J);
      p->mem_loc.push_back(loc);
      loc += pat->blk_dim[J];
    }
    // member indices in ascending molecule order (the gather and scatter search them)
    std::vector<int32_t> srt(order.size());
    for (size_t a = 0; a < srt.size(); ++a) srt[a] = (int32_t)a;
    std::sort(srt.begin(), srt.end(), [&](int32_t x, int32_t y) { return order[x] < order[y]; });
    p->mem_srt.insert(p->mem_srt.end(), srt.begin(), srt.end());
    d.n = loc;
    d.npad = (loc + PAD - 1) / PAD * PAD;
    d.own_lo = p->mem_loc[d.mem_off + own_mem];
    d.m = 0;
    for (const int k : grp) d.m += pat->blk_dim[k];
    if (d.m > MAX_OWN || d.nmem > 1024 || d.npad > 8192)
      return bad(NOLSM_EINVAL,
                 "nolsm_plan_create: submatrix " + std::to_string(i) + " (molecule " +
                     std::to_string(d.mol) + ") exceeds limits (own columns " +
                     std::to_string(d.m) + " <= " + std::to_string(MAX_OWN) + ", members " +
                     std::to_string(d.nmem) + " <= 1024, n " + std::to_string(d.n) + " <= 8192)");
    // the 256 x 128 tiles (tile list 1) iterate on the k-blocked layout
    d.kb = (!literal && d.npad >= big_min) ? 1 : 0;
    p->maxmem = std::max(p->maxmem, d.nmem);
    p->max_npad = std::max(p->max_npad, d.npad);
    p->max_m = std::max(p->max_m, d.m);
  }
  // tiles of the symmetric sign-iteration products: upper triangle; small
  // submatrices use 128 x 128 tiles, the rest 256 x 128 (FP16/BF16) or 128 x 128 (FP32).  Executed flops skip the
  // 32 x 32 blocks that lie entirely in the padding.
  // list 0: small submatrices, 128 x 128 tiles; list 1: large, 256 x 128 tiles (rows x
  // columns; kept when the tile reaches the upper triangle, 2 ti <= tj); list 2: large,
  // 128 x 128 tiles (FP32); list 3: every submatrix, every 128 x 128 tile (not only the
  // upper triangle); lists 4 and 5: every submatrix in 256 x 128 tiles, all of them
  // (4) and the upper triangle (5), for the split-FP16 set-up products
  for (int list = 0; list < NTILELIST; ++list) {
    const int TR = (list == 1 || list >= 4) ? 256 : 128, TC = 128;
    const bool every = list == 3 || list == 4;
    for (int i = 0; i < K; ++i) {
      const int np = p->desc[i].npad;
      if (list < 3 && (np >= big_min) != (list != 0)) continue;
      const int ntr = (np + TR - 1) / TR, ntc = (np + TC - 1) / TC;
      for (int ti = 0; ti < ntr; ++ti)
        for (int tj = 0; tj < ntc; ++tj) {
          if (!every && TR * ti > TC * tj + TC - 1) continue;    // below the diagonal
          p->tiles.push_back(Tile{i, ti, tj, 0});
          const double rows = std::min(TR, np - ti * TR), cols = std::min(TC, np - tj * TC);
          if (list < 2) p->gemm_flop += 2.0 * rows * cols * (double)np;
        }
    }
    p->list_end[list] = (int32_t)p->tiles.size();
  }
  // table buffer: descriptors, member lists, tile lists, per-submatrix state
  off = 0;
  p->off_desc = off;
  off = align256(off + sizeof(SubDesc) * (size_t)K);
  p->off_mem_mol = off;
  off = align256(off + sizeof(int32_t) * p->mem_mol.size());
  p->off_mem_loc = off;
  off = align256(off + sizeof(int32_t) * p->mem_loc.size());
  p->off_mem_srt = off;
  off = align256(off + sizeof(int32_t) * p->mem_srt.size());
  p->off_tiles = off;
  off = align256(off + sizeof(Tile) * p->tiles.size());
  p->off_state = off;
  off = align256(off + sizeof(SubState) * (size_t)K);
  p->tab_bytes = std::max<size_t>(off, 256);
  // workspace: a fixed header shared by every plan bound to the workspace (the
  // executed-flop counter), then the per-submatrix arenas.  The H arena holds the
  // FP32 M_k (4 npad^2 bytes; FP64 T_k(H0) first with the FP32 set-up products,
  // 8 npad^2), the S arena T_k(S), then L^-1 (FP64).  For persist plans these two
  // arenas are laid out in the plan's own buffer instead.
  off = 0;
  p->off_counter = off;
  off = align256(off + sizeof(unsigned long long) + 2 * sizeof(unsigned));
  size_t poff = 0;
  for (int i = 0; i < K; ++i) {
    SubDesc &d = p->desc[i];
    const size_t np = (size_t)d.npad;
    const size_t hbytes = ((setup_fp32 || literal) ? 8 : 4) * np * np;   // FP64 H first
    size_t &o = persist ? poff : off;
    d.off_h = (int64_t)o;
    o = align256(o + hbytes);
    d.off_s = (int64_t)o;
    o = align256(o + 8 * np * np);
    d.off_lo = (int64_t)off;
    off = align256(off + 3 * 4 * np * np);
    d.off_diag = (int64_t)off;
    off = align256(off + 8 * 2 * np * NB);
    d.off_panel = (int64_t)off;
    off = align256(off + 4 * (size_t)NPANEL * np * d.m);
    d.off_dcol = (int64_t)off;
    off = align256(off + 8 * np * d.m);
  }
  p->bytes = off;
  p->persist_bytes = poff;
  *out = p;
  return NOLSM_OK;
}

void nolsm_plan_destroy(nolsm_plan *p) { delete p; }

size_t nolsm_plan_workspace_bytes(const nolsm_plan *p) { return p ? p->bytes : 0; }

size_t nolsm_plan_table_bytes(const nolsm_plan *p) { return p ? p->tab_bytes : 0; }

size_t nolsm_plan_persist_bytes(const nolsm_plan *p) { return p ? p->persist_bytes : 0; }

static nolsm_status bind_impl(nolsm_plan *p, void *tables, size_t table_bytes, void *workspace,
                              size_t bytes, void *persist, size_t persist_bytes, hipStream_t s);

nolsm_status nolsm_plan_bind(nolsm_plan *p, void *tables, size_t table_bytes, void *workspace,
                             size_t bytes, hipStream_t s) {
  if (p && p->persist)
    return fail(NOLSM_EINVAL, "nolsm_plan_bind: the plan keeps its set-up in a buffer of its "
                              "own (use nolsm_plan_bind_persist)");
  return bind_impl(p, tables, table_bytes, workspace, bytes, nullptr, 0, s);
}

nolsm_status nolsm_plan_bind_persist(nolsm_plan *p, void *tables, size_t table_bytes,
                                     void *workspace, size_t bytes, void *persist,
                                     size_t persist_bytes, hipStream_t s) {
  if (p && !p->persist)
    return fail(NOLSM_EINVAL, "nolsm_plan_bind_persist: the plan was created with persist = 0");
  if (p && !persist) return fail(NOLSM_EINVAL, "nolsm_plan_bind_persist: null persist buffer");
  return bind_impl(p, tables, table_bytes, workspace, bytes, persist, persist_bytes, s);
}

static nolsm_status bind_impl(nolsm_plan *p, void *tables, size_t table_bytes, void *workspace,
                              size_t bytes, void *persist, size_t persist_bytes, hipStream_t s) {
  if (!p || !tables || !workspace) return fail(NOLSM_EINVAL, "nolsm_plan_bind: null argument");
  if (table_bytes < p->tab_bytes)
    return fail(NOLSM_EWORKSPACE, "nolsm_plan_bind: table buffer %zu bytes < %zu needed",
                table_bytes, p->tab_bytes);
  if (bytes < p->bytes)
    return fail(NOLSM_EWORKSPACE, "nolsm_plan_bind: workspace %zu bytes < %zu needed", bytes,
                p->bytes);
  if (persist_bytes < p->persist_bytes)
    return fail(NOLSM_EWORKSPACE, "nolsm_plan_bind_persist: persist buffer %zu bytes < %zu needed",
                persist_bytes, p->persist_bytes);
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) || (reinterpret_cast<uintptr_t>(tables) & 255) ||
      (reinterpret_cast<uintptr_t>(persist) & 255))
    return fail(NOLSM_EWORKSPACE, "nolsm_plan_bind: buffers must be 256-byte aligned");
  char *tab = static_cast<char *>(tables);
  char *ws = static_cast<char *>(workspace);
  char *pb = static_cast<char *>(persist);
  const bool same_tables = tab == p->tab && (!p->persist || (ws == p->tab_ws && pb == p->persist_buf));
  // a persist plan keeps its set-up across binds while its own buffers stay the same
  const bool keep_setup = p->persist && same_tables && p->bound;
  if (!same_tables) {
    // first bind to this table buffer (or, for a persist plan, to this pair of
    // workspace and persist buffers): upload the tables and clear the state
    p->tab = nullptr;
    hipError_t e = hipSuccess;
    std::vector<SubDesc> dev_desc;
    const SubDesc *src = p->desc.data();
    if (p->persist && p->K > 0) {
      // every kernel addresses arenas from the workspace base: the persistent ones
      // sit at a fixed signed distance from it
      const int64_t delta = (int64_t)(reinterpret_cast<intptr_t>(pb) - reinterpret_cast<intptr_t>(ws));
      dev_desc = p->desc;
      for (SubDesc &d : dev_desc) {
        d.off_h += delta;
        d.off_s += delta;
      }
      src = dev_desc.data();
    }
    if (p->K > 0) {
      e = hipMemcpyAsync(tab + p->off_desc, src, sizeof(SubDesc) * p->K,
                         hipMemcpyHostToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(tab + p->off_mem_mol, p->mem_mol.data(),
                           sizeof(int32_t) * p->mem_mol.size(), hipMemcpyHostToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(tab + p->off_mem_loc, p->mem_loc.data(),
                           sizeof(int32_t) * p->mem_loc.size(), hipMemcpyHostToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(tab + p->off_mem_srt, p->mem_srt.data(),
                           sizeof(int32_t) * p->mem_srt.size(), hipMemcpyHostToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(tab + p->off_tiles, p->tiles.data(), sizeof(Tile) * p->tiles.size(),
                           hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipMemsetAsync(tab + p->off_state, 0, sizeof(SubState) * p->K, s);
      // the host copies must stay alive until the copies complete
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) return fail(NOLSM_EHIP, "nolsm_plan_bind: %s", hipGetErrorString(e));
    p->tab = tab;
    p->tab_ws = ws;
    p->persist_buf = pb;
  }
  if (!keep_setup) {
    p->setup_done = false;      // the workspace may have served another plan since
    p->scale_ready = false;
  }
  p->ws = ws;
  p->bound = true;
  return NOLSM_OK;
}

nolsm_status nolsm_plan_query(const nolsm_plan *p, int32_t i, nolsm_sub_info *info) {
  if (!p || !info || i < 0 || i >= p->K) return fail(NOLSM_EINVAL, "nolsm_plan_query: bad index");
  const SubDesc &d = p->desc[i];
  info->n = d.n;
  info->npad = d.npad;
  info->mol = d.mol;
  info->m = d.m;
  info->own_lo = d.own_lo;
  info->nmem = d.nmem;
  info->ngrp = d.ngrp;
  info->own_mem = d.own_mem;
  info->off_h = d.off_h;
  info->off_s = d.off_s;
  info->off_lo = d.off_lo;
  info->off_dcol = d.off_dcol;
  return NOLSM_OK;
}

#define PLAN_PTRS                                                                          \
  const SubDesc *desc = reinterpret_cast<const SubDesc *>(p->tab + p->off_desc);           \
  const int32_t *mem_mol = reinterpret_cast<const int32_t *>(p->tab + p->off_mem_mol);     \
  const int32_t *mem_loc = reinterpret_cast<const int32_t *>(p->tab + p->off_mem_loc);     \
  const int32_t *mem_srt = reinterpret_cast<const int32_t *>(p->tab + p->off_mem_srt);     \
  const Tile *tiles = reinterpret_cast<const Tile *>(p->tab + p->off_tiles);               \
  SubState *st = reinterpret_cast<SubState *>(p->tab + p->off_state);                      \
  (void)desc; (void)mem_mol; (void)mem_loc; (void)mem_srt; (void)tiles; (void)st;

static TileSet tile_set(const nolsm_plan *p, const Tile *tiles) {
  TileSet ts;
  for (int l = 0; l < NTILELIST; ++l) {
    const int b = l ? p->list_end[l - 1] : 0;
    ts.t[l] = tiles + b;
    ts.n[l] = p->list_end[l] - b;
  }
  ts.flop_units = reinterpret_cast<unsigned long long *>(p->ws + p->off_counter);
  ts.fb_count = reinterpret_cast<unsigned *>(p->ws + p->off_counter + sizeof(unsigned long long));
  ts.fb_live = ts.fb_count + 1;
  return ts;
}

nolsm_status nolsm_build_submatrices(nolsm_plan *p, const nolsm_pattern *pat, const double *H_val,
                                     const double *S_val, hipStream_t s) {
  if (!p || !pat || !H_val || !S_val) return fail(NOLSM_EINVAL, "nolsm_build_submatrices: null argument");
  if (!p->bound) return fail(NOLSM_EINVAL, "nolsm_build_submatrices: plan not bound");
  if (pat->nmol != p->nmol) return fail(NOLSM_EINVAL, "nolsm_build_submatrices: pattern mismatch");
  if (p->K == 0) return NOLSM_OK;
  PLAN_PTRS
  const int ev = p->log.begin(T_GATHER, s);
  launch_gather(desc, p->K, p->maxmem, mem_mol, mem_loc, mem_srt, pat, H_val, S_val,
                !(p->setup_fp32 || p->literal), p->ws, s);
  p->log.end(ev, s);
  p->setup_done = false;
  p->scale_ready = false;
  return hip_check("nolsm_build_submatrices");
}

nolsm_status nolsm_sign_batched(nolsm_plan *p, double mu, const nolsm_schedule *sched,
                                nolsm_stats *stats, hipStream_t s) {
  if (!p) return fail(NOLSM_EINVAL, "nolsm_sign_batched: null plan");
  if (!std::isfinite(mu)) return fail(NOLSM_EINVAL, "nolsm_sign_batched: mu not finite");
  // the schedule is checked before the plan's buffers (nothing is enqueued either way)
  nolsm_schedule sch;
  if (sched) {
    sch = *sched;
    if (sch.nphase < 1 || sch.nphase > 4) return fail(NOLSM_EINVAL, "nolsm_sign_batched: nphase");
    const bool scaled = sch.lower != nullptr || sch.lower_log10 != nullptr;
    for (int q = 0; q < sch.nphase; ++q) {
      nolsm_phase &ph = sch.phase[q];
      if (ph.prec < 0 || ph.prec > 2 || ph.iters < 0 || ph.iters > 1000 || ph.extra < 0 ||
          !(ph.tol >= 0.0f))
        return fail(NOLSM_EINVAL, "nolsm_sign_batched: bad phase %d", q);
      if (ph.order == 0) ph.order = 2;
      if (ph.order != 2 && ph.order != 3)
        return fail(NOLSM_EINVAL, "nolsm_sign_batched: phase %d order must be 0, 2 or 3", q);
      if (ph.order == 3 && scaled)
        return fail(NOLSM_EINVAL,
                    "nolsm_sign_batched: phase %d: the order-3 step is unscaled (no lower bounds)",
                    q);
    }
    if (sch.panel_steps < 0 || sch.panel_steps > 2)
      return fail(NOLSM_EINVAL, "nolsm_sign_batched: panel_steps must be 0..2");
    if (sch.fallback_iters < 0 || sch.fallback_iters > 1000)
      return fail(NOLSM_EINVAL, "nolsm_sign_batched: fallback_iters");
  } else {
    std::memset(&sch, 0, sizeof sch);
    sch.nphase = 1;
    sch.phase[0].prec = NOLSM_PREC_FP32;
    sch.phase[0].iters = 100;
    sch.phase[0].tol = 1.0e-3f;
    sch.phase[0].extra = 2;
    sch.phase[0].order = 2;
    sch.panel_steps = 0;
    sch.fallback_iters = 0;
  }
  if (!p->bound) return fail(NOLSM_EINVAL, "nolsm_sign_batched: plan not bound");
  if (p->literal) {
    for (int q = 0; q < sch.nphase; ++q) {
      if (sch.phase[q].order == 3)
        return fail(NOLSM_EINVAL, "nolsm_sign_batched: the literal form runs Newton-Schulz "
                                  "steps only (phase %d has order 3)", q);
      if (sch.phase[q].prec != sch.phase[0].prec)
        return fail(NOLSM_EINVAL, "nolsm_sign_batched: the literal form runs every phase in one "
                                  "precision (phase %d differs)", q);
    }
  }
  if (p->K == 0) return NOLSM_OK;
  PLAN_PTRS
  int ev;
  const TileSet ts = tile_set(p, tiles);
  if (!p->setup_done) {
    ev = p->log.begin(T_SETUP, s);
    launch_setup(desc, st, p->K, p->max_npad, ts, p->setup_fp32, !p->factor_fp64, p->literal,
                 p->ws, s);
    p->log.end(ev, s);
    p->setup_done = true;
    p->scale_ready = false;
  }
  ev = p->log.begin(T_SIGN, s);
  const bool have_scale = p->scale_ready && p->scale_mu == mu;
  launch_sign(desc, st, p->K, p->max_npad, ts, p->ws, mu, sch, have_scale, &p->log,
              p->gemm_flop, p->literal, s);
  const nolsm_phase &lastph = sch.phase[sch.nphase - 1];
  launch_final_status(st, p->K, (lastph.tol > 0.0f && sch.fallback_iters == 0) ? 1 : 0, s);
  launch_trace_x(desc, st, p->K, p->ws, s);
  p->log.end(ev, s);
  ev = p->log.begin(T_PANEL, s);
  launch_density_columns(desc, st, p->K, p->max_npad, p->max_m, p->ws, sch.panel_steps,
                         p->literal, s);
  p->log.end(ev, s);
  if (stats) launch_stats(desc, st, p->K, stats, s);
  return hip_check("nolsm_sign_batched");
}

nolsm_status nolsm_setup_batched(nolsm_plan *p, hipStream_t s) {
  if (!p) return fail(NOLSM_EINVAL, "nolsm_setup_batched: null plan");
  if (!p->bound) return fail(NOLSM_EINVAL, "nolsm_setup_batched: plan not bound");
  if (p->K == 0) return NOLSM_OK;
  PLAN_PTRS
  const int ev = p->log.begin(T_SETUP, s);
  launch_setup(desc, st, p->K, p->max_npad, tile_set(p, tiles), p->setup_fp32, !p->factor_fp64,
               p->literal, p->ws, s);
  p->log.end(ev, s);
  p->setup_done = true;
  p->scale_ready = false;
  return hip_check("nolsm_setup_batched");
}

nolsm_status nolsm_features(nolsm_plan *p, double mu, float *feat, hipStream_t s) {
  if (!p || !feat) return fail(NOLSM_EINVAL, "nolsm_features: null argument");
  if (!p->bound) return fail(NOLSM_EINVAL, "nolsm_features: plan not bound");
  if (!std::isfinite(mu)) return fail(NOLSM_EINVAL, "nolsm_features: mu not finite");
  if (p->K == 0) return NOLSM_OK;
  if (!p->setup_done) {
    const nolsm_status r = nolsm_setup_batched(p, s);
    if (r != NOLSM_OK) return r;
  }
  PLAN_PTRS
  launch_features(desc, st, p->K, p->max_npad, p->ws, mu, feat, s);
  p->scale_ready = true;              // the descriptors include the Gershgorin bounds
  p->scale_mu = mu;
  return hip_check("nolsm_features");
}

nolsm_status nolsm_scatter_density(nolsm_plan *p, const nolsm_pattern *pat, double *D_val,
                                   const double *H_val, const double *S_val, nolsm_stats *stats,
                                   hipStream_t s) {
  if (!p || !pat || !D_val || !H_val || !S_val)
    return fail(NOLSM_EINVAL, "nolsm_scatter_density: null argument");
  if (!p->bound) return fail(NOLSM_EINVAL, "nolsm_scatter_density: plan not bound");
  if (pat->nmol != p->nmol) return fail(NOLSM_EINVAL, "nolsm_scatter_density: pattern mismatch");
  if (p->K == 0) return NOLSM_OK;
  PLAN_PTRS
  const int ev = p->log.begin(T_SCATTER, s);
  launch_scatter(desc, st, p->K, p->maxmem, mem_mol, mem_loc, mem_srt, pat, D_val, H_val, S_val,
                 p->ws, stats, s);
  p->log.end(ev, s);
  return hip_check("nolsm_scatter_density");
}

nolsm_status nolsm_energy(const nolsm_pattern *pat, int32_t nmol, const double *D_val,
                          const double *H_val, const double *S_val, double *col_traces,
                          double *out2, hipStream_t s) {
  if (!pat || !D_val || !H_val || !S_val || !col_traces || !out2 || nmol < 0 || nmol != pat->nmol)
    return fail(NOLSM_EINVAL, "nolsm_energy: bad argument");
  launch_energy(pat, nmol, D_val, H_val, S_val, col_traces, out2, s);
  return hip_check("nolsm_energy");
}

nolsm_status nolsm_energy_noalloc(const nolsm_pattern *pat, int32_t nmol, const double *D_val,
                                  const double *H_val, const double *S_val, double *out2,
                                  hipStream_t s) {
  if (!pat || !D_val || !H_val || !S_val || !out2 || nmol < 0 || nmol != pat->nmol)
    return fail(NOLSM_EINVAL, "nolsm_energy_noalloc: bad argument");
  if (nmol > NOLSM_ENERGY_NOALLOC_MAXMOL)
    return fail(NOLSM_EINVAL, "nolsm_energy_noalloc: nmol = %d exceeds the limit %d (use nolsm_energy)",
                nmol, NOLSM_ENERGY_NOALLOC_MAXMOL);
  double *col = nullptr;
  const hipError_t e = energy_scratch_ptr(&col);
  if (e != hipSuccess)
    return fail(NOLSM_EHIP, "nolsm_energy_noalloc: scratch address: %s", hipGetErrorString(e));
  launch_energy(pat, nmol, D_val, H_val, S_val, col, out2, s);
  return hip_check("nolsm_energy_noalloc");
}

nolsm_status nolsm_plan_set_timing(nolsm_plan *p, int enable) {
  if (!p) return fail(NOLSM_EINVAL, "nolsm_plan_set_timing: null plan");
  p->log.on = enable != 0;
  return NOLSM_OK;
}

nolsm_status nolsm_plan_get_timings(nolsm_plan *p, nolsm_timings *out, int reset) {
  if (!p || !out) return fail(NOLSM_EINVAL, "nolsm_plan_get_timings: null argument");
  p->log.collect();
  unsigned long long units = 0;
  if (p->bound && p->K > 0) {
    hipError_t e = hipMemcpy(&units, p->ws + p->off_counter, sizeof units, hipMemcpyDeviceToHost);
    if (e == hipSuccess && reset) e = hipMemset(p->ws + p->off_counter, 0, sizeof units);
    if (e != hipSuccess) return fail(NOLSM_EHIP, "nolsm_plan_get_timings: %s", hipGetErrorString(e));
  }
  p->log.gemm_flop = (double)units * FLOP_UNIT;
  out->ms_gather = p->log.ms[T_GATHER];
  out->ms_setup = p->log.ms[T_SETUP];
  out->ms_sign = p->log.ms[T_SIGN];
  out->ms_gemm = p->log.ms[T_GEMM];
  out->ms_panel = p->log.ms[T_PANEL];
  out->ms_scatter = p->log.ms[T_SCATTER];
  out->n_gemm = p->log.n_gemm;
  out->gemm_flop = p->log.gemm_flop;
  if (reset) {
    for (double &m : p->log.ms) m = 0.0;
    p->log.n_gemm = 0;
    p->log.gemm_flop = 0.0;
  }
  return hip_check("nolsm_plan_get_timings");
}

nolsm_status nolsm_mu_search_init(nolsm_mu_search *m, double n_target, double mu_lo, double mu_hi,
                                  double tol, int32_t max_iter) {
  if (!m) return fail(NOLSM_EINVAL, "nolsm_mu_search_init: null argument");
  if (!std::isfinite(n_target) || !std::isfinite(mu_lo) || !std::isfinite(mu_hi) ||
      !std::isfinite(tol) || !(mu_lo < mu_hi) || tol < 0.0 || max_iter < 1 || max_iter > 1000)
    return fail(NOLSM_EINVAL, "nolsm_mu_search_init: need finite values, mu_lo < mu_hi, tol >= 0, "
                              "1 <= max_iter <= 1000");
  std::memset(m, 0, sizeof *m);
  m->n_target = n_target;
  m->tol = tol;
  m->lo = mu_lo;
  m->hi = mu_hi;
  m->mu = 0.5 * (mu_lo + mu_hi);
  m->last_n = NAN;
  m->max_iter = max_iter;
  return NOLSM_OK;
}

nolsm_status nolsm_mu_search_update(nolsm_mu_search *m, double n_at_mu) {
  if (!m) return fail(NOLSM_EINVAL, "nolsm_mu_search_update: null argument");
  if (m->done != 0) return fail(NOLSM_EINVAL, "nolsm_mu_search_update: the search has ended");
  if (!std::isfinite(n_at_mu))
    return fail(NOLSM_EINVAL, "nolsm_mu_search_update: electron count not finite");
  m->last_n = n_at_mu;
  ++m->iters;
  if (n_at_mu < m->n_target - m->tol) {
    m->lo = m->mu;
  } else if (n_at_mu > m->n_target + m->tol) {
    m->hi = m->mu;
  } else {
    m->done = 1;                 // m->mu is the result
    return NOLSM_OK;
  }
  if (m->iters >= m->max_iter) {
    m->done = -1;                // m->mu stays the last trial
    return NOLSM_OK;
  }
  m->mu = 0.5 * (m->lo + m->hi);
  return NOLSM_OK;
}

nolsm_status nolsm_check(nolsm_plan *p, hipStream_t s) {
  if (!p || !p->bound) return fail(NOLSM_EINVAL, "nolsm_check: plan not bound");
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(NOLSM_EHIP, "nolsm_check: %s", hipGetErrorString(e));
  std::vector<SubState> host(p->K);
  if (p->K > 0) {
    e = hipMemcpy(host.data(), p->tab + p->off_state, sizeof(SubState) * p->K, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(NOLSM_EHIP, "nolsm_check: %s", hipGetErrorString(e));
  }
  int nspd = 0, nconv = 0, first = -1;
  for (int i = 0; i < p->K; ++i) {
    if (host[i].status == NOLSM_ENOTSPD) { ++nspd; if (first < 0) first = i; }
    if (host[i].status == NOLSM_ENOCONV) { ++nconv; if (first < 0) first = i; }
  }
  if (nspd) return fail(NOLSM_ENOTSPD, "%d submatrices not positive definite (first: batch index %d)", nspd, first);
  if (nconv) return fail(NOLSM_ENOCONV, "%d submatrices did not converge (first: batch index %d)", nconv, first);
  return NOLSM_OK;
}

}  // extern "C"
