// C ABI of libhankel: argument checking, workspace layout and the launch
// sequence of the path (load -> panels of Algorithm 1 -> Algorithm 4 -> block ->
// eigen-step).  All device memory is the caller's.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hl_kernels.hpp"
#include "hl_host.hpp"

using namespace hl;

struct hl_ctx {
  int device = 0;
  int timing = 0;
  int karatsuba = -1;  // Schur update form for MFMA shapes: -1 by precision, else Karatsuba levels (0 = digit product)
  int eig_maxit = 0;   // iteration limit of the eigen-step per block (0: the default)
  // pivot lookahead of the MFMA form: a second stream (default priority) and
  // the events joining it to the caller's
  hipStream_t aux = nullptr;
  hipEvent_t ev_col = nullptr, ev_piv = nullptr;
  hl_timing_t t{};
  std::vector<hipEvent_t> pool;
  size_t used = 0;
};

static thread_local std::string g_err;

namespace hl {
hl_status fail(hl_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}
}  // namespace hl

#define HIPCHK(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) return fail(HL_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

extern "C" const char* hl_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// shape -> dims and workspace layout
namespace hl {

hl_status make_dims(const hl_shape* sh, Dims* dm) {
  if (!sh) return fail(HL_EINVAL, "null shape");
  if (sh->N < 1 || sh->N > 8192) return fail(HL_EINVAL, "N=%d out of range [1, 8192]", sh->N);
  if (sh->k < 1 || sh->k > sh->N || sh->k > 32) return fail(HL_EINVAL, "k=%d out of range", sh->k);
  if (sh->prec_bits % 128 || sh->prec_bits < 256 || sh->prec_bits > kMaxPrec)
    return fail(HL_EINVAL, "prec_bits=%d must be a multiple of 128 in [256, %d]", sh->prec_bits, kMaxPrec);
  if (sh->exp_block < 1) return fail(HL_EINVAL, "exp_block must be >= 1");
  if (sh->form != HL_FORM_MFMA8 && sh->form != HL_FORM_VALU) return fail(HL_EINVAL, "bad form");
  dm->N = sh->N;
  dm->NT = (sh->N + 31) / 32 * 32;
  dm->nt = dm->NT / 32;
  dm->P = sh->prec_bits;
  dm->nl = sh->prec_bits / 32;
  dm->nw = 2 * dm->nl;
  dm->S = 4 * dm->nl;
  dm->E = sh->exp_block;
  dm->k = sh->k;
  dm->W = 2 * sh->prec_bits - 4;
  dm->Sk0 = (dm->S + 255) / 256 * 256;
  // Karatsuba levels offered: every level splits the Sk0-digit strings on whole
  // slabs; beyond the default level only while the products fit kKaraExtraBytes
  dm->kara = 0;
  if (sh->form == HL_FORM_MFMA8)
    for (int lv = 1; lv <= KA_MAX_LEVELS; ++lv) {
      const size_t tri = (size_t)dm->nt * (dm->nt + 1) / 2;
      const size_t bytes = (size_t)kara_products(lv) * tri * tile_words(kara_nwp(dm->Sk0, lv)) * 4;
      if (lv > kara_auto_level(dm->P) && bytes > kKaraExtraBytes) break;
      dm->kara = lv;
    }
  return HL_OK;
}

static size_t al(size_t x) { return (x + 255) / 256 * 256; }

Layout make_layout(const Dims& dm) {
  Layout L{};
  size_t off = 0;
  L.status = off;
  off += 256;
  L.tiles = off;
  off += al((size_t)dm.nt * (dm.nt + 1) / 2 * tile_words(dm.nw) * 4);
  L.upanel = off;
  off += al((size_t)16 * dm.NT * dm.nl * 4);
  L.omega_stride = dm.nl + 4;
  L.omega = off;
  off += al((size_t)dm.N * L.omega_stride * 4);
  // int8 digit panels for the MFMA form, padded by kDigitPad slices at both ends
  L.digit_slices = dm.S + 2 * kDigitPad;
  L.bdig = off;
  off += al((size_t)L.digit_slices * dm.NT * 16);
  L.udig = off;
  off += al((size_t)L.digit_slices * dm.NT * 16);
  L.carry = off;
  {
    // one carry slot of 1024 entries per work item (tile x limb range) of an
    // MFMA launch; the range count is chosen within this capacity
    const size_t tri = (size_t)dm.nt * (dm.nt + 1) / 2;
    const size_t rect = (size_t)dm.nt * ((dm.k + 31) / 32);
    const size_t tiles = tri > rect ? tri : rect;
    const size_t useful = tiles * (size_t)(kMaxRanges < dm.nl / 2 ? kMaxRanges : dm.nl / 2);
    L.carry_tiles = 16384 + tiles < useful ? 16384 + tiles : useful;
    for (int lv = 1; lv <= dm.kara; ++lv) {
      // the Karatsuba forms have 3^lv products per tile
      const size_t np = kara_products(lv);
      const size_t ntbp = (size_t)kara_nwp(dm.Sk0, lv) / 4;
      const size_t kuse = np * tri * (kMaxRanges < ntbp ? kMaxRanges : ntbp);
      const size_t kt = 16384 + np * tri < kuse ? 16384 + np * tri : kuse;
      if (kt > L.carry_tiles) L.carry_tiles = kt;
    }
    off += al(L.carry_tiles * 1024 * 8);
  }
  // block: per pair and row chunk partial sums of 3nl + 8 limbs
  const int npairs = dm.k * (dm.k + 1) / 2;
  L.blk_stride = 3 * dm.nl + 16;
  L.blk_chunks = (dm.N + kBlockRows - 1) / kBlockRows;
  L.blk_part = off;
  off += al((size_t)npairs * L.blk_chunks * L.blk_stride * 4);
  L.blk_sum = off;
  off += al((size_t)npairs * (L.blk_stride + 64) * 4);
  L.eig = off;
  off += al(eig_ws_bytes(dm));
  {
    const size_t ns = 4 * (size_t)dm.nl + 4;
    L.adj_y = off;
    off += al((size_t)dm.k * dm.nl * 4);
    L.adj_yc = off;
    off += al((size_t)dm.k * dm.nl * 4);
    L.adj_ysq = off;
    off += al(((size_t)2 * dm.nl + 2) * 4);
    L.adj_z = off;
    off += al((size_t)dm.NT * dm.nl * 4);
    L.adj_wp = off;
    off += 256;
    L.adj_part = off;
    off += al((size_t)dm.N * ns * 4);
    L.adj_col = off;
    off += al(ns * 8);
    L.adj_tot = off;
    off += al(ns * 4);
  }
  {
    // Toeplitz-form updates: up to 16 factor columns, max(16, k) target columns
    const size_t cols = dm.k > 16 ? dm.k : 16;
    L.colprod_ld = 2 * dm.nl + 4;
    L.blk_ny = 2 * dm.nl + 4;
    L.blk_nm = 3 * dm.nl + 4;
    // users: trailing-matrix targets (nw limbs, up to NT rows), the column
    // products (one column of colprod_ld limbs), the block sums (32 rows of b
    // digits of 2 nl + 1 limbs, k columns of blk_nm limbs)
    const size_t b1 = (size_t)16 * dm.NT * tp_bstride(4 * (2 * dm.nl + 1));  // b rows up to 2 nl + 1 limbs
    const size_t b2 = (size_t)16 * 32 * tp_bstride(4 * (2 * dm.nl + 1));
    L.toep_b_bytes = b1 > b2 ? b1 : b2;
    L.toep_b = off;
    off += al(L.toep_b_bytes);
    L.toep_u_bytes = (size_t)16 * cols * tp_ustride(dm.S + 4);
    L.toep_u = off;
    off += al(L.toep_u_bytes);
    size_t items = (size_t)dm.nt * cols * tp_ranges(dm.nw);
    const size_t i2 = (size_t)dm.nt * tp_ranges(L.colprod_ld), i3 = (size_t)dm.k * tp_ranges(L.blk_nm);
    if (i2 > items) items = i2;
    if (i3 > items) items = i3;
    L.toep_carry_words = items * 32;
    L.toep_carry = off;
    off += al(L.toep_carry_words * 8);
    L.colprod = off;
    off += al((size_t)dm.NT * L.colprod_ld * 4);
    L.blk_y = off;
    off += al((size_t)dm.k * dm.NT * L.blk_ny * 4);
    L.blk_m = off;
    off += al((size_t)dm.k * dm.k * L.blk_nm * 4);
    L.adj_nr = 3 * dm.nl + 4;
    L.adj_da = off;
    off += al((size_t)16 * dm.N * dm.nw * 4);
    L.adj_r = off;
    off += al((size_t)dm.N * L.adj_nr * 4);
  }
  if (dm.kara) {
    L.kara_tiles = (size_t)dm.nt * (dm.nt + 1) / 2;
    size_t words = 0;
    for (int lv = 1; lv <= dm.kara; ++lv) {
      L.kara_pan_slices[lv] = kara_leaf_digits(dm.Sk0, lv) + 2 * kDigitPad;
      L.kara_pan_bytes[lv] = al((size_t)L.kara_pan_slices[lv] * dm.NT * 16);
      L.kara_pan[lv] = off;
      off += 2 * kara_products(lv) * L.kara_pan_bytes[lv];
      const size_t w = kara_products(lv) * L.kara_tiles * tile_words(kara_nwp(dm.Sk0, lv));
      if (w > words) words = w;
    }
    L.kara_prod = off;
    off += al(words * 4);
  }
  L.total = off;
  return L;
}

}  // namespace hl

// Toeplitz-form update over the workspace's digit and carry regions
ToepArgs hl::toep_args(const UpdArgs& g, const Layout& L, char* base, const Dims& dm) {
  ToepArgs a{};
  a.g = g;
  a.bd = (int8_t*)(base + L.toep_b);
  a.ud = (int8_t*)(base + L.toep_u);
  a.carry = (long long*)(base + L.toep_carry);
  a.bd_bytes = L.toep_b_bytes;
  a.ud_bytes = L.toep_u_bytes;
  a.carry_words = L.toep_carry_words;
  a.S = dm.S;
  a.NT = dm.NT;
  return a;
}

extern "C" hl_status hl_get_sizes(const hl_shape* sh, hl_sizes* out) {
  Dims dm;
  hl_status s = make_dims(sh, &dm);
  if (s != HL_OK) return s;
  if (!out) return fail(HL_EINVAL, "null output");
  Layout L = make_layout(dm);
  memset(out, 0, sizeof *out);
  out->workspace_bytes = L.total;
  out->d_words = (size_t)dm.N * dm.nw;
  out->l_words = (size_t)dm.N * dm.NT * dm.nl;
  out->x_words = (size_t)dm.NT * dm.k * dm.nl;
  out->blk_words = (size_t)dm.k * dm.k * dm.nl;
  out->nl = dm.nl;
  out->NT = dm.NT;
  out->trail_offset = L.tiles;
  out->trail_bytes = (size_t)dm.nt * (dm.nt + 1) / 2 * tile_words(dm.nw) * 4;
  out->diag_offset = L.eig;
  return HL_OK;
}

extern "C" hl_status hl_create(hl_ctx** ctx, int device) {
  if (!ctx) return fail(HL_EINVAL, "null ctx");
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(HL_EINVAL, "device %d of %d", device, n);
  HIPCHK(hipSetDevice(device));
  HIPCHK(noalloc_init(device));  // device address of hl_lambda_min_noalloc's scratch
  hl_ctx* c = new hl_ctx();
  c->device = device;
  *ctx = c;
  return HL_OK;
}

extern "C" hl_status hl_destroy(hl_ctx* ctx) {
  if (!ctx) return HL_OK;
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->ev_col) (void)hipEventDestroy(ctx->ev_col);
  if (ctx->ev_piv) (void)hipEventDestroy(ctx->ev_piv);
  if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
  delete ctx;
  return HL_OK;
}

extern "C" hl_status hl_set_eig_maxit(hl_ctx* ctx, int32_t maxit) {
  if (!ctx) return fail(HL_EINVAL, "null ctx");
  if (maxit < 0) return fail(HL_EINVAL, "maxit=%d must be >= 0", maxit);
  ctx->eig_maxit = maxit;
  return HL_OK;
}

int hl::ctx_eig_maxit(const hl_ctx* ctx) { return ctx ? ctx->eig_maxit : 0; }

extern "C" hl_status hl_set_timing(hl_ctx* ctx, int enable) {
  if (!ctx) return fail(HL_EINVAL, "null ctx");
  ctx->timing = enable;
  return HL_OK;
}

extern "C" hl_status hl_set_karatsuba(hl_ctx* ctx, int32_t mode) {
  if (!ctx) return fail(HL_EINVAL, "null ctx");
  if (mode < -1 || mode > KA_MAX_LEVELS) return fail(HL_EINVAL, "karatsuba mode %d not in [-1, %d]", mode, KA_MAX_LEVELS);
  ctx->karatsuba = mode;
  return HL_OK;
}

extern "C" hl_status hl_get_timing(hl_ctx* ctx, hl_timing_t* out) {
  if (!ctx || !out) return fail(HL_EINVAL, "null argument");
  *out = ctx->t;
  return HL_OK;
}

// event helpers: pairs recorded around stages, summed at the next sync
namespace hl {
struct Stamp {
  hl_ctx* ctx;
  hipStream_t s;
  int slot;
  hipEvent_t a = nullptr, b = nullptr;
  Stamp(hl_ctx* c, hipStream_t st, int sl) : ctx(c), s(st), slot(sl) {
    if (!ctx->timing) return;
    if (ctx->used + 2 > ctx->pool.size()) {
      for (int j = 0; j < 64; ++j) {
        hipEvent_t e;
        (void)hipEventCreate(&e);
        ctx->pool.push_back(e);
      }
    }
    a = ctx->pool[ctx->used++];
    b = ctx->pool[ctx->used++];
    (void)hipEventRecord(a, s);
  }
  void end() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    ctx->t.ms[slot] += ms;
    ctx->used -= 2;
    a = nullptr;
  }
};
}  // namespace hl

static hl_status check_ws(const Layout& L, void* ws, size_t ws_bytes) {
  if (!ws) return fail(HL_EINVAL, "null workspace");
  if (ws_bytes < L.total) return fail(HL_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, L.total);
  return HL_OK;
}

// ---------------------------------------------------------------------------
// A narrow update of the MFMA form: few entries take one workgroup each (the
// workgroup MFMA product), the others the Toeplitz-form kernel; same bits.
// Used for the updates inside a 16-row block of the triangular solve (at most
// 15 x k entries) and of the adjoint's back substitution (at most 15); the
// in-panel updates of the factorisation measured faster in the Toeplitz form
// even when few.
static hipError_t launch_upd_narrow(const UpdArgs& g, const Layout& L, char* base, const Dims& dm, hipStream_t st) {
  if (g.r_hi <= g.r_lo || g.c_hi <= g.c_lo || g.npan <= 0) return hipSuccess;
  if ((size_t)(g.r_hi - g.r_lo) * (g.c_hi - g.c_lo) <= kUpdWgEntries) {
    const hipError_t e = launch_upd_wg(g, st);
    if (e != hipErrorInvalidValue) return e;
  }
  return launch_upd_toep(toep_args(g, L, base, dm), st);
}

// the context's second stream (default priority) and its events, made once
static hipError_t ensure_aux(hl_ctx* ctx) {
  if (ctx->aux) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_col, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_piv, hipEventDisableTiming);
  return e;
}

extern "C" hl_status hl_factor(hl_ctx* ctx, const hl_shape* sh, const uint32_t* mu, const int64_t* mu_exp,
                               int32_t w, void* ws, size_t ws_bytes, const hl_factor_t* out, void* stream) {
  return hl_factor_cols(ctx, sh, mu, mu_exp, w, ws, ws_bytes, out, 0, sh ? sh->N : 0, stream);
}

extern "C" hl_status hl_factor_cols(hl_ctx* ctx, const hl_shape* sh, const uint32_t* mu, const int64_t* mu_exp,
                                    int32_t w, void* ws, size_t ws_bytes, const hl_factor_t* out,
                                    int32_t col_begin, int32_t col_end, void* stream) {
  if (!ctx) return fail(HL_EINVAL, "null ctx");
  Dims dm;
  hl_status s = make_dims(sh, &dm);
  if (s != HL_OK) return s;
  if (!mu || !mu_exp || w < 1) return fail(HL_EINVAL, "bad moments");
  if (!out || !out->d || !out->h || !out->s || !out->l) return fail(HL_EINVAL, "null factor output");
  Layout L = make_layout(dm);
  if ((s = check_ws(L, ws, ws_bytes)) != HL_OK) return s;
  if (col_begin < 0 || col_end > dm.N || col_begin > col_end || col_begin % 16 || (col_end % 16 && col_end != dm.N))
    return fail(HL_EINVAL, "column range [%d, %d) must be panel aligned", col_begin, col_end);
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  DevStatus* dst = (DevStatus*)(base + L.status);
  u32* A = (u32*)(base + L.tiles);
  u32* up = (u32*)(base + L.upanel);
  u32* omega = (u32*)(base + L.omega);
  ctx->t = hl_timing_t{};
  int kara_lv = ctx->karatsuba >= 0 ? ctx->karatsuba : kara_auto_level(dm.P);
  if (kara_lv > dm.kara) kara_lv = dm.kara;

  Stamp total(ctx, st, 7);
  if (col_begin == 0) {
  Stamp ld(ctx, st, 5);
  HIPCHK(launch_fill((u32*)dst, 64, 0u, st));
  HIPCHK(launch_fill(out->l, (size_t)dm.N * dm.NT * dm.nl, 0u, st));
  if (sh->form == HL_FORM_MFMA8) {
    // zero digit slices (the padding outside [0, S) must read as zero)
    HIPCHK(launch_fill((u32*)(base + L.bdig), (size_t)L.digit_slices * dm.NT * 4, 0u, st));
    HIPCHK(launch_fill((u32*)(base + L.udig), (size_t)L.digit_slices * dm.NT * 4, 0u, st));
    for (int lv = 1; lv <= dm.kara; ++lv)
      HIPCHK(launch_fill((u32*)(base + L.kara_pan[lv]), 2 * kara_products(lv) * L.kara_pan_bytes[lv] / 4, 0u, st));
  }
  HIPCHK(launch_scales(mu, mu_exp, w, dm.N, dm.E, out->s, dst, st));
  HIPCHK(launch_load(mu, mu_exp, w, out->s, dm, A, dst, st));
  ld.end();
  }

  const size_t ldb = (size_t)dm.NT * dm.nl;
  // MFMA form: pivot i + 1 runs on the aux stream while column i's step and
  // in-panel update run on the caller's; it forms b_{i+1} u_{i+1} of column i
  // itself and subtracts it, so that update leaves out the diagonal row i + 1
  const bool look = sh->form == HL_FORM_MFMA8;
  if (look) HIPCHK(ensure_aux(ctx));
  for (int i0 = col_begin; i0 < col_end; i0 += 16) {
    const int npan = dm.N - i0 < 16 ? dm.N - i0 : 16;
    Stamp pn(ctx, st, 1);
    for (int il = 0; il < npan; ++il) {
      const int i = i0 + il;
      if (!look || il == 0) {
        HIPCHK(launch_pivot(A, dm, i, out->d, out->h, omega, L.omega_stride, dst, st));
      } else {
        HIPCHK(hipStreamWaitEvent(st, ctx->ev_piv, 0));
      }
      if (look && il + 1 < npan) {
        // pivot i + 1 needs pivot i and row i + 1 as the previous columns'
        // updates left it: it forms row i + 1's factors of column i itself and
        // runs beside this column's step and update
        HIPCHK(hipEventRecord(ctx->ev_col, st));
        HIPCHK(hipStreamWaitEvent(ctx->aux, ctx->ev_col, 0));
        HIPCHK(launch_pivot(A, dm, i + 1, out->d, out->h, omega, L.omega_stride, dst, ctx->aux, nullptr, nullptr,
                            1));
        HIPCHK(hipEventRecord(ctx->ev_piv, ctx->aux));
      }
      if (sh->form == HL_FORM_MFMA8) {
        u32* ucol = up + (size_t)il * ldb;
        u32* P = (u32*)(base + L.colprod);
        // one launch with a workgroup MFMA product per row; where its LDS does
        // not fit, col_u -> Toeplitz product -> col_fin
        const hipError_t ec = launch_col_m(A, dm, i, i0, out->h, omega, L.omega_stride, ucol,
                                           out->l + (size_t)i * ldb, dst, st);
        if (ec != hipErrorInvalidValue) {
          HIPCHK(ec);
        } else {
          HIPCHK(launch_col_u(A, dm, i, i0, out->h, ucol, dst, st));
          // P_r = u_r w_i for rows i+1 .. N-1: rank 1 against the single column w_i
          UpdArgs g{};
          g.A = P;
          g.nw = L.colprod_ld;
          g.nl = dm.nl;
          g.Bop = ucol;
          g.Uop = omega + (size_t)i * L.omega_stride;
          g.npan = 1;
          g.r_lo = i + 1;
          g.r_hi = dm.N;
          g.c_lo = 0;
          g.c_hi = 1;
          g.st = dst;
          ToepArgs ta = toep_args(g, L, base, dm);
          ta.nlb = dm.nl;
          ta.nlu = dm.nl + 1;  // w_i <= 2^P
          ta.plain = 1;
          ta.ldr = (size_t)L.colprod_ld;
          ta.ldc = 0;
          ta.add = 2;
          HIPCHK(launch_upd_toep(ta, st));
          HIPCHK(launch_col_fin(dm, i, i0, P, L.colprod_ld, out->l + (size_t)i * ldb, dst, st));
        }
      } else {
        HIPCHK(launch_col(A, dm, i, i0, out->h, omega, L.omega_stride, up + (size_t)il * ldb,
                          out->l + (size_t)i * ldb, dst, st));
      }
      if (il + 1 < npan) {
        UpdArgs g{};
        g.A = A;
        g.tri = 1;
        g.nw = dm.nw;
        g.nl = dm.nl;
        g.Bop = out->l + (size_t)i * ldb;
        g.ldb = ldb;
        g.Uop = up + (size_t)il * ldb;
        g.ldu = ldb;
        g.npan = 1;
        g.r_lo = look ? i + 2 : i + 1;
        g.r_hi = dm.N;
        g.c_lo = i + 1;
        g.c_hi = i0 + npan;
        g.st = dst;
        if (sh->form == HL_FORM_MFMA8) {
          HIPCHK(launch_upd_toep(toep_args(g, L, base, dm), st));
        } else {
          HIPCHK(launch_upd_valu(g, st));
        }
      }
    }
    pn.end();
    if (i0 + npan < dm.N) {
      Stamp su(ctx, st, 0);
      UpdArgs g{};
      g.A = A;
      g.tri = 1;
      g.nw = dm.nw;
      g.nl = dm.nl;
      g.Bop = out->l + (size_t)i0 * ldb;
      g.ldb = ldb;
      g.Uop = up;
      g.ldu = ldb;
      g.npan = npan;
      g.r_lo = i0 + npan;
      g.r_hi = dm.N;
      g.c_lo = i0 + npan;
      g.c_hi = dm.N;
      g.st = dst;
      hipError_t e;
      if (sh->form == HL_FORM_MFMA8) {
        MfmaArgs m{};
        m.g = g;
        m.bdig = (int8_t*)(base + L.bdig);
        m.udig = (int8_t*)(base + L.udig);
        m.slices = L.digit_slices;
        m.pad = kDigitPad;
        m.S = dm.S;
        m.NT = dm.NT;
        m.carry = (long long*)(base + L.carry);
        m.max_ranges = kMaxRanges;
        m.carry_tiles = L.carry_tiles;
        m.timing = ctx->timing ? &ctx->t : nullptr;
        m.u_rows = dm.NT;
        if (kara_lv > 0) {
          KaraArgs ka{};
          ka.m = m;
          ka.m.S = dm.Sk0;  // the Karatsuba form's digit strings (zero digits above S)
          ka.levels = kara_lv;
          for (int lv = 1; lv <= kara_lv; ++lv) {
            ka.pan[lv] = (int8_t*)(base + L.kara_pan[lv]);
            ka.pan_stride[lv] = L.kara_pan_bytes[lv];
            ka.pan_slices[lv] = L.kara_pan_slices[lv];
          }
          ka.Sk = kara_leaf_digits(dm.Sk0, kara_lv);
          ka.kslices = ka.Sk + 2 * kDigitPad;
          ka.prod = (u32*)(base + L.kara_prod);
          ka.nwp = kara_nwp(dm.Sk0, kara_lv);
          ka.prod_tiles = L.kara_tiles;
          e = launch_upd_kara(ka, st);
        } else {
          e = launch_upd_mfma(m, st);
        }
      } else {
        e = launch_upd_valu(g, st);
      }
      HIPCHK(e);
      ctx->t.launches[0] += 1;
      const double rows = dm.N - (i0 + npan);
      ctx->t.schur_limb_macs += (double)npan * rows * (rows + 1) / 2 * (double)dm.nl * dm.nl;
      su.end();
    }
  }
  total.end();
  return HL_OK;
}

extern "C" hl_status hl_sync(hl_ctx* ctx, void* ws, void* stream, int32_t* index) {
  if (!ctx || !ws) return fail(HL_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  unsigned long long v = 0;
  HIPCHK(hipMemcpy(&v, ws, 8, hipMemcpyDeviceToHost));
  const int code = (int)(v >> 32);
  const int idx = (int)(v & 0xffffffffu);
  if (index) *index = idx;
  if (code) return fail((hl_status)code, "device status %d at index %d", code, idx);
  return HL_OK;
}

// ---------------------------------------------------------------------------
extern "C" hl_status hl_debug_mul(const uint32_t* a, int32_t na, const uint32_t* b, int32_t nb, uint32_t* out,
                                  int32_t nout, void* stream) {
  if (!a || !b || !out || na < 1 || nb < 1 || nout < 1) return fail(HL_EINVAL, "bad debug_mul args");
  HIPCHK(launch_debug_mul(a, na, b, nb, out, nout, (hipStream_t)stream));
  return HL_OK;
}

extern "C" hl_status hl_debug_mul_wg(const uint32_t* a, int32_t na, const uint32_t* b, int32_t nb, uint32_t* out,
                                     int32_t nout, int32_t threads, void* stream) {
  if (!a || !b || !out || na < 1 || nb < 1 || nout < 1 || (threads != 256 && threads != 1024))
    return fail(HL_EINVAL, "bad debug_mul_wg args");
  HIPCHK(launch_debug_mul_wg(a, na, b, nb, out, nout, threads, (hipStream_t)stream));
  return HL_OK;
}

extern "C" hl_status hl_debug_valu_peak(int32_t mode, int32_t blocks, int32_t iters, uint64_t* sink, void* stream) {
  if ((mode != 0 && mode != 1) || blocks < 1 || iters < 1 || !sink) return fail(HL_EINVAL, "bad debug_valu_peak args");
  HIPCHK(launch_valu_peak(mode, blocks, iters, (u64*)sink, (hipStream_t)stream));
  return HL_OK;
}

extern "C" hl_status hl_debug_recip(const uint32_t* d, int32_t nd, int32_t P, uint32_t* omega, int32_t* h,
                                    void* stream) {
  if (!d || !omega || !h || P % 128 || P < 256 || P > kMaxPrec || nd < 1 || nd > 2 * (P / 32))
    return fail(HL_EINVAL, "bad debug_recip args");
  HIPCHK(launch_debug_recip(d, nd, P, omega, P / 32 + 4, h, (hipStream_t)stream));
  return HL_OK;
}

// ---------------------------------------------------------------------------
extern "C" hl_status hl_inv_block(hl_ctx* ctx, const hl_shape* sh, const hl_factor_t* f, void* ws, size_t ws_bytes,
                                  uint32_t* x, uint32_t* blk, int64_t* blk_exp, void* stream) {
  if (!ctx) return fail(HL_EINVAL, "null ctx");
  Dims dm;
  hl_status s = make_dims(sh, &dm);
  if (s != HL_OK) return s;
  if (!f || !f->d || !f->h || !f->s || !f->l || !x || !blk || !blk_exp) return fail(HL_EINVAL, "null argument");
  Layout L = make_layout(dm);
  if ((s = check_ws(L, ws, ws_bytes)) != HL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  DevStatus* dst = (DevStatus*)(base + L.status);
  u32* ACC = (u32*)(base + L.tiles);  // the trailing matrix is finished: reuse as accumulators
  u32* omega = (u32*)(base + L.omega);
  const size_t ldb = (size_t)dm.NT * dm.nl;
  const size_t ldx = (size_t)dm.k * dm.nl;

  Stamp ts(ctx, st, 2);
  HIPCHK(launch_fill(ACC, (size_t)dm.nt * tile_words(dm.nw), 0u, st));
  HIPCHK(launch_fill(x, (size_t)dm.NT * dm.k * dm.nl, 0u, st));  // rows N .. NT-1 stay zero
  for (int R0 = 0; R0 < dm.N; R0 += 16) {
    const int nb = dm.N - R0 < 16 ? dm.N - R0 : 16;
    for (int j = 0; j < nb; ++j) {
      const int r = R0 + j;
      HIPCHK(launch_trsm_row(ACC, dm, r, f->s, f->h, x, dst, st));
      if (j + 1 < nb) {
        UpdArgs g{};
        g.A = ACC;
        g.tri = 0;
        g.ntc = 1;
        g.nw = dm.nw;
        g.nl = dm.nl;
        g.Bop = f->l + (size_t)r * ldb;
        g.ldb = ldb;
        g.Uop = x + (size_t)r * ldx;
        g.ldu = ldx;
        g.npan = 1;
        g.r_lo = r + 1;
        g.r_hi = R0 + nb;
        g.c_lo = 0;
        g.c_hi = dm.k;
        g.st = dst;
        if (sh->form == HL_FORM_MFMA8) {
          HIPCHK(launch_upd_narrow(g, L, base, dm, st));
        } else {
          HIPCHK(launch_upd_valu(g, st));
        }
      }
    }
    if (R0 + nb < dm.N) {
      UpdArgs g{};
      g.A = ACC;
      g.tri = 0;
      g.ntc = 1;
      g.nw = dm.nw;
      g.nl = dm.nl;
      g.Bop = f->l + (size_t)R0 * ldb;
      g.ldb = ldb;
      g.Uop = x + (size_t)R0 * ldx;
      g.ldu = ldx;
      g.npan = nb;
      g.r_lo = R0 + nb;
      g.r_hi = dm.N;
      g.c_lo = 0;
      g.c_hi = dm.k;
      g.st = dst;
      if (sh->form == HL_FORM_MFMA8) {
        // k <= 32 target columns: the Toeplitz form keeps every MFMA column busy
        HIPCHK(launch_upd_toep(toep_args(g, L, base, dm), st));
      } else {
        HIPCHK(launch_upd_valu(g, st));
      }
    }
  }
  ts.end();
  Stamp tb(ctx, st, 3);
  if (sh->form == HL_FORM_MFMA8) {
    // M_ab = sum_r (x_rb w_r) x_ra: y by products, the sum over r as Toeplitz
    // MFMA GEMMs of rank 16 accumulated into M (rows b, columns a <= b)
    u32* Y = (u32*)(base + L.blk_y);
    u32* M = (u32*)(base + L.blk_m);
    // The rank-16 launches over r leave half the GPU idle (k rows per 32-row
    // item), so the odd row chunks run on the second stream into an
    // accumulator and Toeplitz scratch of their own, carved from the
    // trailing-matrix region (dead once the solve above has run); the gather
    // adds the two accumulators.
    const size_t mwords = (size_t)dm.k * dm.k * L.blk_nm;
    const size_t o_bd = al(mwords * 4), o_ud = o_bd + al(L.toep_b_bytes), o_cy = o_ud + al(L.toep_u_bytes);
    const bool two = dm.N > 16 && o_cy + L.toep_carry_words * 8 <= L.upanel - L.tiles;
    char* t2 = base + L.tiles;
    u32* M2 = two ? (u32*)t2 : nullptr;
    HIPCHK(launch_fill(M, mwords, 0u, st));
    if (two) {
      HIPCHK(ensure_aux(ctx));
      HIPCHK(launch_fill(M2, mwords, 0u, st));
    }
    HIPCHK(launch_block_y(x, dm, omega, L.omega_stride, Y, L.blk_ny, dst, st));
    if (two) {
      HIPCHK(hipEventRecord(ctx->ev_col, st));
      HIPCHK(hipStreamWaitEvent(ctx->aux, ctx->ev_col, 0));
    }
    for (int r0 = 0; r0 < dm.N; r0 += 16) {
      UpdArgs g{};
      g.A = M;
      g.tri = 1;
      g.nw = L.blk_nm;
      g.nl = dm.nl;
      g.Bop = Y + (size_t)r0 * L.blk_ny;
      g.ldb = L.blk_ny;
      g.rsb = (size_t)dm.NT * L.blk_ny;
      g.Uop = x + (size_t)r0 * ldx;
      g.ldu = ldx;
      g.npan = dm.N - r0 < 16 ? dm.N - r0 : 16;
      g.r_lo = 0;
      g.r_hi = dm.k;
      g.c_lo = 0;
      g.c_hi = dm.k;
      g.st = dst;
      ToepArgs ta = toep_args(g, L, base, dm);
      ta.NT = 32;  // b digit rows: the k <= 32 columns of y
      ta.nlb = 2 * dm.nl + 1;
      ta.nlu = dm.nl;
      ta.ucs = (size_t)dm.nl;
      ta.plain = 1;
      ta.ldr = (size_t)dm.k * L.blk_nm;
      ta.ldc = (size_t)L.blk_nm;
      ta.add = 1;
      const bool odd = two && ((r0 / 16) & 1);
      if (odd) {
        ta.g.A = M2;
        ta.bd = (int8_t*)(t2 + o_bd);
        ta.ud = (int8_t*)(t2 + o_ud);
        ta.carry = (long long*)(t2 + o_cy);
      }
      HIPCHK(launch_upd_toep(ta, odd ? ctx->aux : st));
    }
    if (two) {
      HIPCHK(hipEventRecord(ctx->ev_piv, ctx->aux));
      HIPCHK(hipStreamWaitEvent(st, ctx->ev_piv, 0));
    }
    u32* part = (u32*)(base + L.blk_part);
    HIPCHK(launch_block_gather(M, M2, L.blk_nm, dm, part, L.blk_stride, dst, st));
    HIPCHK(launch_block_sums(dm, f->s, part, L.blk_stride, 1, (u32*)(base + L.blk_sum), L.blk_stride + 64, blk,
                             blk_exp, dst, st));
  } else {
    HIPCHK(launch_block(x, dm, omega, L.omega_stride, f->s, (u32*)(base + L.blk_part), L.blk_stride, L.blk_chunks,
                        kBlockRows, (u32*)(base + L.blk_sum), L.blk_stride + 64, blk, blk_exp, dst, st));
  }
  tb.end();
  return HL_OK;
}

// value (sign, exponent, mantissa top limbs) of a device float -> double and P-bit mantissa
static double fp_to_double(int sign, long e, const std::vector<uint32_t>& m) {
  // m: NWM limbs, top bit of m.back() set; value = (M / 2^(32 NWM)) 2^e
  const size_t n = m.size();
  const uint64_t top = ((uint64_t)m[n - 1] << 32) | m[n - 2];
  double v = std::ldexp((double)(top >> 11), (int)(e - 53));
  return sign ? -v : v;
}

extern "C" hl_status hl_lambda_min(hl_ctx* ctx, const hl_shape* sh, const uint32_t* blk, const int64_t* blk_exp,
                                   void* ws, size_t ws_bytes, uint32_t* lam_mant, uint32_t* lam_mant_km1,
                                   hl_lambda_t* out, void* stream) {
  if (!ctx) return fail(HL_EINVAL, "null ctx");
  Dims dm;
  hl_status s = make_dims(sh, &dm);
  if (s != HL_OK) return s;
  if (!blk || !blk_exp || !out) return fail(HL_EINVAL, "null argument");
  Layout L = make_layout(dm);
  if ((s = check_ws(L, ws, ws_bytes)) != HL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  DevStatus* dst = (DevStatus*)(base + L.status);
  void* ews = base + L.eig;
  Stamp te(ctx, st, 4);
  HIPCHK(ensure_aux(ctx));
  HIPCHK(launch_eig_host(blk, dm, ews, dst, st, ctx->aux, ctx->eig_maxit));
  te.end();
  int32_t idx = 0;
  if ((s = hl_sync(ctx, ws, stream, &idx)) != HL_OK) return s;
  int64_t bexp = 0;
  HIPCHK(hipMemcpy(&bexp, blk_exp, 8, hipMemcpyDeviceToHost));
  return read_lambda(dm, ews, bexp, lam_mant, lam_mant_km1, out);
}

// one multiprecision result of the eigen-step as a double and (optionally) its
// top nl limbs on the device; *e_out = exponent of those limbs
static hl_status read_fp(const Dims& dm, int* hdr, u32* mant, int64_t bexp, double* v_out, int64_t* e_out,
                         uint32_t* dst) {
  const int NWM = dm.nl + 4;
  int h2[2];
  std::vector<uint32_t> m(NWM);
  HIPCHK(hipMemcpy(h2, hdr, 8, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(m.data(), mant, (size_t)NWM * 4, hipMemcpyDeviceToHost));
  const long e = (long)h2[1] - bexp;
  *v_out = h2[0] == 2 ? 0.0 : fp_to_double(h2[0], e, m);
  if (e_out) *e_out = e - 32L * dm.nl;
  if (dst) HIPCHK(hipMemcpy(dst, m.data() + (NWM - dm.nl), (size_t)dm.nl * 4, hipMemcpyHostToDevice));
  return HL_OK;
}

extern "C" hl_status hl_lambda_next(hl_ctx* ctx, const hl_shape* sh, const uint32_t* blk, const int64_t* blk_exp,
                                    void* ws, size_t ws_bytes, int32_t count, uint32_t* mant, uint32_t* mant_km1,
                                    hl_lambda_j_t* out, void* stream) {
  if (!ctx) return fail(HL_EINVAL, "null ctx");
  Dims dm;
  hl_status s = make_dims(sh, &dm);
  if (s != HL_OK) return s;
  if (!blk || !blk_exp || !out) return fail(HL_EINVAL, "null argument");
  if (count < 1 || count > 2) return fail(HL_EINVAL, "count=%d: 1 or 2 further eigenvalues", count);
  if (dm.k < count + 2) return fail(HL_EINVAL, "k=%d: lambda_%d with its estimate needs k >= %d", dm.k, count + 1,
                                    count + 2);
  Layout L = make_layout(dm);
  if ((s = check_ws(L, ws, ws_bytes)) != HL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  DevStatus* dst = (DevStatus*)(base + L.status);
  void* ews = base + L.eig;
  HIPCHK(launch_eig_next(blk, dm, ews, count, dst, st));
  int32_t idx = 0;
  if ((s = hl_sync(ctx, ws, stream, &idx)) != HL_OK) return s;
  int64_t bexp = 0;
  HIPCHK(hipMemcpy(&bexp, blk_exp, 8, hipMemcpyDeviceToHost));
  for (int j = 1; j <= count; ++j) {
    hl_lambda_j_t& o = out[j - 1];
    memset(&o, 0, sizeof o);
    o.j = j + 1;
    int* hdr = nullptr;
    u32* m = nullptr;
    eig_next_refs(dm, ews, 2 * j, false, &hdr, &m);
    if ((s = read_fp(dm, hdr, m, bexp, &o.lambda, &o.exp, mant ? mant + (size_t)(j - 1) * dm.nl : nullptr)) != HL_OK)
      return s;
    eig_next_refs(dm, ews, 2 * j + 1, false, &hdr, &m);
    if ((s = read_fp(dm, hdr, m, bexp, &o.lambda_km1, &o.exp_km1,
                     mant_km1 ? mant_km1 + (size_t)(j - 1) * dm.nl : nullptr)) != HL_OK)
      return s;
    eig_next_refs(dm, ews, 2 * j, true, &hdr, &m);
    if ((s = read_fp(dm, hdr, m, bexp, &o.trunc, nullptr, nullptr)) != HL_OK) return s;
    int it[2];
    HIPCHK(hipMemcpy(&it[0], eig_iter_ref(ews, 2 * j), 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&it[1], eig_iter_ref(ews, 2 * j + 1), 4, hipMemcpyDeviceToHost));
    o.iterations = it[0] + it[1];
  }
  return HL_OK;
}

namespace hl {
// host readback of the eigen-step's results (after the stream has finished)
hl_status read_lambda(const Dims& dm, void* ews, int64_t bexp, uint32_t* lam_mant, uint32_t* lam_mant_km1,
                      hl_lambda_t* out) {
  const int NWM = dm.nl + 4;
  memset(out, 0, sizeof *out);
  for (int which = 0; which < 3; ++which) {
    if (which > 0 && dm.k < 2) {
      if (which == 1) out->lambda1_km1 = std::nan("");
      if (which == 2) out->trunc = std::nan("");
      continue;
    }
    int* hdr = nullptr;
    u32* mant = nullptr;
    eig_result_refs(dm, ews, which, &hdr, &mant);
    int h2[2];
    std::vector<uint32_t> m(NWM);
    HIPCHK(hipMemcpy(h2, hdr, 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(m.data(), mant, (size_t)NWM * 4, hipMemcpyDeviceToHost));
    double v;
    long e = (long)h2[1] - bexp;  // lambda_1 = (1 / lambda_max(blk)) 2^-blk_exp
    if (h2[0] == 2) {
      v = 0.0;
    } else {
      v = fp_to_double(h2[0], e, m);
    }
    uint32_t* dstm = which == 0 ? lam_mant : (which == 1 ? lam_mant_km1 : nullptr);
    if (which == 0) {
      out->lambda1 = v;
      out->exp = e - 32L * dm.nl;
    } else if (which == 1) {
      out->lambda1_km1 = v;
      out->exp_km1 = e - 32L * dm.nl;
    } else {
      out->trunc = v;
    }
    if (dstm) HIPCHK(hipMemcpy(dstm, m.data() + (NWM - dm.nl), (size_t)dm.nl * 4, hipMemcpyHostToDevice));
  }
  int fl[16];
  HIPCHK(hipMemcpy(fl, ews, sizeof fl, hipMemcpyDeviceToHost));
  out->iterations = fl[1] + fl[9];
  return HL_OK;
}
}  // namespace hl

// ---------------------------------------------------------------------------
// a nonnegative little-endian limb array as m 2^e, m in [1/2, 1) (m = 0 for 0)
static double limbs_to_double(const std::vector<uint32_t>& x, long* e) {
  int top = (int)x.size() - 1;
  while (top >= 0 && x[top] == 0) --top;
  if (top < 0) {
    *e = 0;
    return 0.0;
  }
  uint64_t hi = ((uint64_t)x[top] << 32) | (top >= 1 ? x[top - 1] : 0u);
  const uint32_t lo = top >= 2 ? x[top - 2] : 0u;
  int lz = 0;
  while (!(hi >> 63)) {
    hi = (hi << 1) | ((lo >> (31 - lz)) & 1u);
    ++lz;
  }
  // value = hi 2^(32 (top - 1) - lz) up to the bits below
  *e = 32L * (top - 1) - lz + 64;
  return std::ldexp((double)(hi >> 11), -53);
}

static void limbs_negate(std::vector<uint32_t>& x) {
  uint64_t c = 1;
  for (auto& v : x) {
    const uint64_t t = (uint64_t)(uint32_t)~v + c;
    v = (uint32_t)t;
    c = t >> 32;
  }
}

extern "C" hl_status hl_lambda_grad(hl_ctx* ctx, const hl_shape* sh, const hl_factor_t* f, const uint32_t* x,
                                    const int64_t* blk_exp, const uint32_t* dmu, const int64_t* dmu_exp,
                                    const int32_t* dmu_neg, int32_t w, void* ws, size_t ws_bytes, uint32_t* z,
                                    hl_grad_t* out, void* stream) {
  if (!ctx) return fail(HL_EINVAL, "null ctx");
  Dims dm;
  hl_status s = make_dims(sh, &dm);
  if (s != HL_OK) return s;
  if (!f || !f->d || !f->h || !f->s || !f->l || !x || !blk_exp || !dmu || !dmu_exp || !dmu_neg || !out)
    return fail(HL_EINVAL, "null argument");
  if (w < 1) return fail(HL_EINVAL, "w must be >= 1");
  Layout L = make_layout(dm);
  if ((s = check_ws(L, ws, ws_bytes)) != HL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  DevStatus* dst = (DevStatus*)(base + L.status);
  int32_t idx = 0;
  if ((s = hl_sync(ctx, ws, stream, &idx)) != HL_OK) return s;

  // lambda_1 = (1 / lambda_max(blk)) 2^-blk_exp from the eigen-step
  const int NWM = dm.nl + 4;
  int* rh = nullptr;
  u32* rm = nullptr;
  eig_result_refs(dm, base + L.eig, 0, &rh, &rm);
  int h2[2];
  std::vector<uint32_t> lm(NWM);
  int64_t bexp = 0;
  HIPCHK(hipMemcpy(h2, rh, 8, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(lm.data(), rm, (size_t)NWM * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&bexp, blk_exp, 8, hipMemcpyDeviceToHost));
  if (h2[0] != 0) return fail(HL_EINVAL, "no positive lambda_1 in the workspace: run hl_lambda_min first");
  long le = 0;
  const double lmant = limbs_to_double(lm, &le);   // 1/lambda_max = lmant 2^(le - 32 NWM + h2[1])
  le += (long)h2[1] - 32L * NWM - bexp;             // lambda_1 = lmant 2^le
  const double lam1 = std::ldexp(lmant, (int)le);

  // scales: s0 = min_{m<k} s_m, Q = W - (max_{m<k} s_m + 64), s_max over all rows
  std::vector<int32_t> sv(dm.N);
  HIPCHK(hipMemcpy(sv.data(), f->s, (size_t)dm.N * 4, hipMemcpyDeviceToHost));
  int s0 = sv[0], sk = sv[0], smax = sv[0];
  for (int m = 0; m < dm.k; ++m) {
    s0 = sv[m] < s0 ? sv[m] : s0;
    sk = sv[m] > sk ? sv[m] : sk;
  }
  for (int i = 0; i < dm.N; ++i) smax = sv[i] > smax ? sv[i] : smax;
  const long Q = (long)dm.W - (sk + 64);
  // |v_i| <= |y| lambda_1 / lambda_min(H) ~ |y|, so |z_i| <~ sqrt(k) 2^(s_i - W) / lambda_1;
  // F keeps the largest below 2^(P - 8 - 16)
  const long lg = (long)std::ceil(0.5 * std::log2((double)dm.k) - (std::log2(lmant) + (double)le));
  const long F = (long)dm.P - 8 - ((long)smax - dm.W) - (lg > 0 ? lg : 0) - 16;
  const long eG = F - Q - s0 - 2L * dm.P + 3;

  u32* ACC = (u32*)(base + L.tiles);
  u32* Y = (u32*)(base + L.adj_y);
  u32* Yc = (u32*)(base + L.adj_yc);
  u32* ysq = (u32*)(base + L.adj_ysq);
  u32* Z = (u32*)(base + L.adj_z);
  i64* wp = (i64*)(base + L.adj_wp);
  u32* part = (u32*)(base + L.adj_part);
  unsigned long long* col = (unsigned long long*)(base + L.adj_col);
  u32* tot = (u32*)(base + L.adj_tot);
  const size_t nlz = (size_t)dm.nl;

  Stamp ta(ctx, st, 8);
  HIPCHK(launch_fill(ACC, (size_t)dm.nt * tile_words(dm.nw), 0u, st));
  int* yh = nullptr;
  u32* ym = nullptr;
  eig_vector_refs(dm, base + L.eig, &yh, &ym);
  HIPCHK(launch_adj_y(yh, ym, NWM, dm, f->s, Y, Yc, ysq, dst, st));
  HIPCHK(launch_adj_g(x, Yc, (const u32*)(base + L.omega), L.omega_stride, dm, eG, ACC, dst, st));
  // B^T z = G from the last row up, in blocks of 16 rows
  for (int i0 = (dm.N - 1) / 16 * 16; i0 >= 0; i0 -= 16) {
    const int nb = dm.N - i0 < 16 ? dm.N - i0 : 16;
    for (int i = i0 + nb - 1; i >= i0; --i) {
      HIPCHK(launch_adj_row(ACC, dm, i, f->h, Z, dst, st));
      if (i > i0) {
        // rows [i0, i) of the block: acc_r -= b_ir z_i
        UpdArgs g{};
        g.A = ACC;
        g.tri = 0;
        g.ntc = 1;
        g.nw = dm.nw;
        g.nl = dm.nl;
        g.Bop = f->l + (size_t)i * nlz;
        g.ldb = nlz;
        g.rsb = (size_t)dm.NT * nlz;
        g.Uop = Z + (size_t)i * nlz;
        g.ldu = nlz;
        g.npan = 1;
        g.r_lo = i0;
        g.r_hi = i;
        g.c_lo = 0;
        g.c_hi = 1;
        g.st = dst;
        if (sh->form == HL_FORM_MFMA8) {
          HIPCHK(launch_upd_narrow(g, L, base, dm, st));
        } else {
          HIPCHK(launch_upd_valu(g, st));
        }
      }
    }
    if (i0 > 0) {
      // rows above the block: acc_r -= sum_{i in block} b_ir z_i
      UpdArgs g{};
      g.A = ACC;
      g.tri = 0;
      g.ntc = 1;
      g.nw = dm.nw;
      g.nl = dm.nl;
      g.Bop = f->l + (size_t)i0 * nlz;
      g.ldb = nlz;
      g.rsb = (size_t)dm.NT * nlz;
      g.Uop = Z + (size_t)i0 * nlz;
      g.ldu = nlz;
      g.npan = nb;
      g.r_lo = 0;
      g.r_hi = i0;
      g.c_lo = 0;
      g.c_hi = 1;
      g.st = dst;
      if (sh->form == HL_FORM_MFMA8) {
        HIPCHK(launch_upd_toep(toep_args(g, L, base, dm), st));
      } else {
        HIPCHK(launch_upd_valu(g, st));
      }
    }
  }
  if (sh->form == HL_FORM_MFMA8) {
    // R_i = sum_j da_ij z_j as Toeplitz MFMA GEMMs of rank 16 over j
    u32* DA = (u32*)(base + L.adj_da);
    u32* R = (u32*)(base + L.adj_r);
    HIPCHK(launch_adj_wprime(dmu, dmu_exp, w, dm, f->s, wp, st));
    HIPCHK(launch_fill(R, (size_t)dm.N * L.adj_nr, 0u, st));
    for (int j0 = 0; j0 < dm.N; j0 += 16) {
      const int npan = dm.N - j0 < 16 ? dm.N - j0 : 16;
      HIPCHK(launch_adj_da(dmu, dmu_exp, (const int*)dmu_neg, w, dm, f->s, wp, j0, npan, DA, dm.nw, dst, st));
      UpdArgs g{};
      g.A = R;
      g.nw = L.adj_nr;
      g.nl = dm.nl;
      g.Bop = DA;
      g.ldb = (size_t)dm.N * dm.nw;
      g.rsb = (size_t)dm.nw;
      g.Uop = Z + (size_t)j0 * nlz;
      g.ldu = nlz;
      g.npan = npan;
      g.r_lo = 0;
      g.r_hi = dm.N;
      g.c_lo = 0;
      g.c_hi = 1;
      g.st = dst;
      ToepArgs ta2 = toep_args(g, L, base, dm);
      ta2.nlb = dm.nw;  // |da| < 2^(2P-3)
      ta2.nlu = dm.nl;
      ta2.plain = 1;
      ta2.ldr = (size_t)L.adj_nr;
      ta2.ldc = 0;
      ta2.add = 1;
      HIPCHK(launch_upd_toep(ta2, st));
    }
    HIPCHK(launch_adj_finish(R, L.adj_nr, Z, dm, part, col, tot, dst, st));
  } else {
    HIPCHK(launch_adj_contract(dmu, dmu_exp, (const int*)dmu_neg, w, dm, f->s, wp, Z, part, col, tot, dst, st));
  }
  if (z) HIPCHK(hipMemcpyAsync(z, Z, (size_t)dm.N * nlz * 4, hipMemcpyDeviceToDevice, st));
  ta.end();
  if ((s = hl_sync(ctx, ws, stream, &idx)) != HL_OK) return s;

  const size_t ns = 4 * nlz + 4;
  std::vector<uint32_t> T(ns), q(2 * nlz + 2);
  int64_t Wp = 0;
  HIPCHK(hipMemcpy(T.data(), tot, ns * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(q.data(), ysq, q.size() * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&Wp, wp, 8, hipMemcpyDeviceToHost));
  memset(out, 0, sizeof *out);
  out->lambda1 = lam1;
  out->z_shift = F;
  out->num_offset = L.adj_tot;
  out->num_limbs = (int32_t)ns;
  out->den_offset = L.adj_ysq;
  out->den_limbs = (int32_t)(2 * nlz + 2);
  long qe = 0;
  const double qm = limbs_to_double(q, &qe);
  if (qm == 0.0) return fail(HL_EINVAL, "eigenvector is zero");
  out->ynorm = std::sqrt(qm) * std::ldexp(1.0, (int)(qe / 2 - (dm.P - 3))) * ((qe & 1) ? std::sqrt(2.0) : 1.0);
  if (Wp == LLONG_MAX) return HL_OK;  // dmu = 0
  out->num_shift = 2L * dm.W - Wp - 2 * F + 2L * dm.P - 6;
  const bool neg = (T[ns - 1] >> 31) != 0;
  if (neg) limbs_negate(T);
  long te = 0;
  const double tm = limbs_to_double(T, &te);
  // d lambda_1 = lambda_1^2 2^(2W - W' - 2F + 2P - 6) Tot / sum Y^2
  const long ex = 2 * le + te - qe + 2L * dm.W - Wp - 2 * F + 2L * dm.P - 6;
  const double v = lmant * lmant * tm / qm;
  out->dlambda1 = std::ldexp(neg ? -v : v, (int)(ex < -100000 ? -100000 : (ex > 100000 ? 100000 : ex)));
  return HL_OK;
}

extern "C" hl_status hl_debug_mfma_layout(int32_t* out, void* stream) {
  if (!out) return fail(HL_EINVAL, "null output");
  HIPCHK(launch_mfma_probe(out, (hipStream_t)stream));
  return HL_OK;
}
