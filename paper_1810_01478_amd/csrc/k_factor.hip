// Load of the scaled Hankel matrix and the per-pivot steps of Algorithm 1
// (serial LDL^T, Section 4.3): the pivot, its rounded reciprocal, and the two
// factor columns u (the paper's A_i[j], cut to P bits) and b (the paper's
// B_i[k] = A_i[k] / A_i[i], scaled by 2^h_i).
#include "hl_kernels.hpp"
#include "mp_mfma.hpp"

namespace hl {

// ---------------------------------------------------------------------------
// Row scale exponents: s_j = ceil(t_J / 2), t_J = max_{j in J} bitlen(mu_2j),
// for blocks J of E rows (power-of-two form of the diagonal preconditioner of
// Section 6.2).
__global__ void k_scales(const u32* __restrict__ mu, const i64* __restrict__ mu_exp, int w, int N,
                         int E, i32* __restrict__ s_out, DevStatus* st) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  const int nJ = (N + E - 1) / E;
  if (J >= nJ) return;
  long tJ = LONG_MIN;
  const int j1 = min(N, J * E + E);
  for (int j = J * E; j < j1; ++j) {
    const u32* m = mu + (size_t)(2 * j) * w;
    int top = w - 1;
    while (top >= 0 && m[top] == 0) --top;
    if (top < 0) {
      set_status(st, HL_EINVAL, 2 * j);
      return;
    }
    const long bl = (long)top * 32 + (32 - __clz((int)m[top])) + mu_exp[2 * j];
    tJ = bl > tJ ? bl : tJ;
  }
  const long sJ = -((-tJ) >> 1);  // ceil(tJ / 2), arithmetic shift floors
  for (int j = J * E; j < j1; ++j) s_out[j] = (i32)sJ;
}

// ---------------------------------------------------------------------------
// a_rc = rnd(mu_{r+c} 2^(W - s_r - s_c)) for r >= c (Section 2, eq. matrix);
// entries outside the N x N matrix are zero.  One thread per tile entry.
__global__ void k_load(const u32* __restrict__ mu, const i64* __restrict__ mu_exp, int w,
                       const i32* __restrict__ s, Dims dm, u32* __restrict__ A, DevStatus* st) {
  const size_t t = blockIdx.x;
  // invert t = R (R + 1) / 2 + C by bisection on R
  int lo = 0, hi = dm.nt;  // R in [lo, hi)
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if ((size_t)mid * (mid + 1) / 2 <= t) lo = mid; else hi = mid;
  }
  const int R = lo;
  const int C = (int)(t - (size_t)R * (R + 1) / 2);
  const int r = R * 32 + (threadIdx.x >> 5), c = C * 32 + (threadIdx.x & 31);
  u32* base = A + t * tile_words(dm.nw);
  const int nq = dm.nw / 4;
  if (r >= dm.N || c >= dm.N || c > r) {
    for (int q = 0; q < nq; ++q)
      *(uint4*)(base + in_tile(r, c, 4 * q)) = make_uint4(0, 0, 0, 0);
    return;
  }
  const int m = r + c;
  const u32* M = mu + (size_t)m * w;
  const long sig = mu_exp[m] + (long)dm.W - s[r] - s[c];
  int top = w - 1;
  while (top >= 0 && M[top] == 0) --top;
  const long bl = top < 0 ? 0 : (long)top * 32 + (32 - __clz((int)M[top])) + sig;
  if (bl > (long)dm.W + 1) {
    set_status(st, HL_EOVERFLOW, r);
    return;
  }
  u32 carry = 0;
  if (sig < 0) carry = get_bit(M, w, -sig - 1);  // round half up (M >= 0)
  for (int q = 0; q < nq; ++q) {
    u32 v[4];
    for (int j = 0; j < 4; ++j) {
      const int l = 4 * q + j;
      u32 x = sig >= 0 ? limb_shl(M, w, sig, l) : limb_shr(M, w, -sig, l);
      u64 s2 = (u64)x + carry;
      v[j] = (u32)s2;
      carry = (u32)(s2 >> 32);
    }
    *(uint4*)(base + in_tile(r, c, 4 * q)) = make_uint4(v[0], v[1], v[2], v[3]);
  }
}

// ---------------------------------------------------------------------------
// Pivot reciprocal.  For the pivot d (nw limbs in LDS, positive) computes
//   h = bitlen(d) / 2 and w = rnd(2^(2h+P) / d), the quotient by the whole
//   pivot rounded once (ties away from zero).
// The work runs on d~ = floor(d / 2^m), d cut to its top P + 64 bits
// (m = max(0, bitlen(d) - P - 64)), with the power lowered by m: Newton's
// iteration y <- y + y (1 - delta y) for y ~ 1/delta, delta = d~ / 2^bitlen(d~),
// with the working precision roughly doubled per step, then the remainder
// R~ = 2^(2h+P-m) - Z d~ corrects Z to the exact floor of q~ = 2^(2h+P-m) / d~.
// Since d~ 2^m <= d < (d~ + 1) 2^m and q < 2^(P+1), q~ - 2^-62 < q <= q~, so
// rnd(q) is rnd(q~) or one less, and it can be one less only when q~ lies
// within 2^-62 above a half-integer (2 R~ - d~ < d~ 2^-61).  In that case the
// cut part delta = d mod 2^m decides exactly: with r = Z + 1,
//   (2r - 1) d - 2^(2h+P+1) = (2Z + 1) delta - (2 R~ - d~) 2^m,
// and q < r - 1/2 (round down) exactly when that is positive.
// LDS: 15 (nl + 8) words below the pivot (see pivot_lds_bytes).
struct PivotOut {
  int h;
  int ok;
};

// out = 2^e - T (mod 2^(32n)), T zero-extended from nT; out may be T.  All
// threads of the workgroup; rip as for wg_resolve.
__device__ void wg_sub_from_pow2(long e, const u32* T, int nT, u32* out, int n, u32* rip) {
  wg_resolve(n, [=](int p) -> u64 {
    u64 v = (u64)(~(p < nT ? T[p] : 0u)) + (p == 0 ? 1u : 0u);
    if ((long)p == (e >> 5)) v += (u64)1 << (e & 31);
    return v;
  }, out, rip);
}

// x += d (two's complement add of a sign-extended small signed value), n limbs
__device__ void wg_add_i32(u32* x, int n, int d, u32* rip) {
  const u32 ext = d < 0 ? 0xffffffffu : 0u;
  wg_resolve(n, [=](int p) -> u64 { return (u64)x[p] + (p == 0 ? (u32)d : ext); }, x, rip);
}

constexpr long kPivWaveBits = 2048;  // Newton steps up to this precision run in one wave

// Product for the reciprocal's steps (non-negative operands): the one-workgroup
// MFMA form once the operands are large and its scratch fits in the column-sum
// buffer (cap bytes), else the product scan on the vector ALU.  Same bits.
// lo_limb > 0 (the MFMA form only): limbs below lo_limb need not be formed and
// the limbs from there on may lack the carry out of the part below (see
// wg_mfma_mul); the product scan forms the whole product.
__device__ __forceinline__ void pv_mul(const u32* a, int na, const u32* b, int nb, u32* out, int nout, u32* buf,
                                       size_t cap, int lo_limb = 0) {
  if ((long)na * nb >= 16384 && wm_scratch_bytes(na, nb) <= cap)
    wg_mfma_mul(a, na, b, nb, out, nout, buf, lo_limb);
  else
    g_mul(a, na, b, nb, out, nout, buf);
}

__device__ PivotOut pivot_recip(const u32* d, int nw, int P, u32* omega, int n_omega, u32* lds,
                                int nl) {
  // every thread of the block calls this and every step runs on all waves:
  // the products, the shifts, and the carry chains (wg_resolve)
  PivotOut res{0, 1};
  const int NB = nl + 8;
  u32* D = lds;            // d~
  u32* Y = D + NB;
  u32* Yn = Y + NB;
  u32* dq = Yn + NB;
  u32* Z = dq + NB;
  u32* T = Z + NB;         // 2 NB
  u32* T2 = T + 2 * NB;    // 2 NB
  u32* colbuf = T2 + 2 * NB;  // 6 NB: scratch of the products, and between them of the carry chains
  u32* rip = colbuf;
  const size_t cap = (size_t)6 * NB * 4;
  const int Ld = w_bitlen(d, nw);
  const int h = Ld / 2;
  res.h = h;
  const long m = Ld - (long)P - 64 > 0 ? Ld - (long)P - 64 : 0;
  const int nd = nl + 2;
  wg_shift_right(d, nw, m, D, nd);
  const int LD = w_bitlen(D, nd);
  const long e = 2L * h + P - m;
  const long pf = e - LD + 40;   // final precision of y
  // initial 30-bit estimate from the top 32 bits of D
  if (wave_id() == 0) {
    const u32 dtop = LD >= 32 ? limb_shr(D, nd, LD - 32, 0) : limb_shl(D, nd, 32 - LD, 0);
    const u64 y0 = ((u64)1 << 62) / (u64)dtop;
    if (lane_id() == 0) Y[0] = (u32)y0;
    for (int p2 = 1 + lane_id(); p2 < NB; p2 += WAVE) Y[p2] = 0;
  }
  __syncthreads();
  long p = 30;
  int ny = 1;
  // The steps up to kPivWaveBits of precision, whose operands have at most 66
  // limbs, run in wave 0 alone with the wave's own carry chains (the same
  // arithmetic as the workgroup steps below, without a workgroup barrier per
  // operation); the other waves wait at one barrier.
  __shared__ long wv_p;
  __shared__ int wv_ny, wv_fail;
  if (wave_id() == 0) {
    long pw = p;
    int nyw = ny, fail = 0;
    while (pw < pf) {
      long pn = pf;
      while ((pn + 13) / 2 > pw) pn = (pn + 13) / 2;
      if (pn > kPivWaveBits) break;
      const long q = pn + 8;
      const int nq = (int)(q / 32) + 2;
      w_shift_right(D, nd, LD - q, dq, nq);
      wsync();
      // T = dq Y, then E = 2^(p+q) - T over nT + 1 limbs
      const int nT = nq + nyw, nE = nT + 1;
      w_mul(dq, nq, Y, nyw, T, nT);
      if (lane_id() == 0) T[nT] = 0;
      wsync();
      w_neg(T, nE);
      wsync();
      w_add_word(T, nE, (int)((pw + q) >> 5), 1u << ((pw + q) & 31));
      wsync();
      const bool neg = (T[nE - 1] >> 31) != 0;
      if (neg) {
        w_neg(T, nE);
        wsync();
      }
      int ne = (w_bitlen(T, nE) + 31) / 32;
      if (ne < 1) ne = 1;
      if (ne > nq + 2) {
        fail = 1;
        break;
      }
      const int nT2 = nyw + ne;
      w_mul(Y, nyw, T, ne, T2, nT2);
      wsync();
      const int nyn = (int)((pn + 2) / 32) + 2;
      w_shift_right(Y, nyw, -(pn - pw), Yn, nyn);
      w_shift_right(T2, nT2, 2 * pw + q - pn, Z, nyn);
      wsync();
      if (neg) {
        w_sub(Yn, Z, Y, nyn);
      } else {
        w_add(Yn, nyn, Z, nyn, Y, nyn);
      }
      w_fill(Y + nyn, NB - nyn, 0u);
      wsync();
      nyw = nyn;
      pw = pn;
    }
    if (lane_id() == 0) {
      wv_p = pw;
      wv_ny = nyw;
      wv_fail = fail;
    }
  }
  __syncthreads();
  p = wv_p;
  ny = wv_ny;
  if (wv_fail) res.ok = 0;
  while (p < pf && res.ok) {
    // precisions planned back from pf, each step at most doubling (less 12
    // guard bits): pn is the smallest of pf, c(pf), c(c(pf)), ... above p,
    // c(t) = ceil((t + 12) / 2), so the last step starts near pf / 2
    long pn = pf;
    while ((pn + 13) / 2 > p) pn = (pn + 13) / 2;
    const long q = pn + 8;
    const int nq = (int)(q / 32) + 2;
    // dq = floor(D * 2^(q - LD))
    wg_shift_right(D, nd, LD - q, dq, nq);
    // T = dq * Y, E = 2^(p+q) - T.  A converging step has |E| < 2^(32 (nq + 2))
    // (checked below), so once p + q reaches 32 (nq + 3), E is T's low nq + 3
    // limbs negated, read as a signed number: only those limbs of the product
    // are formed
    const bool short_t = p + q >= 32L * (nq + 3);
    const int nT = short_t ? nq + 3 : nq + ny;
    pv_mul(dq, nq, Y, ny, T, nT, colbuf, cap);
    // E = 2^(p+q) - T  (two's complement over nE limbs)
    const int nE = short_t ? nT : nT + 1;
    wg_sub_from_pow2(p + q, T, nT, T, nE, rip);
    const bool neg = (T[nE - 1] >> 31) != 0;
    __syncthreads();
    if (neg) wg_neg(T, nE, rip);
    // T2 = Y * |E|, then shifted
    int ne = (w_bitlen(T, nE) + 31) / 32;
    if (ne < 1) ne = 1;
    if (ne > nq + 2) {  // |1 - delta y| is not small: the iteration has diverged
      res.ok = 0;
      break;
    }
    // T2 = Y |E|, of which only the bits from 2p + q - pn up are used: the
    // limbs more than two below them are not formed (Z may come out one unit
    // low or high, within the step's guard bits)
    const int nT2 = ny + ne;
    const long zlo = (2 * p + q - pn) / 32 - 2;
    pv_mul(Y, ny, T, ne, T2, nT2, colbuf, cap, zlo > 0 ? (int)zlo : 0);
    const int nyn = (int)((pn + 2) / 32) + 2;
    // Yn = Y << (pn - p);   Z = T2 >> (2p + q - pn)
    wg_shift_right(Y, ny, -(pn - p), Yn, nyn);
    wg_shift_right(T2, nT2, 2 * p + q - pn, Z, nyn);
    if (neg) {
      wg_sub(Yn, Z, Y, nyn, rip);
    } else {
      wg_add(Yn, nyn, Z, nyn, Y, nyn, rip);
    }
    for (int j = nyn + threadIdx.x; j < NB; j += blockDim.x) Y[j] = 0;
    __syncthreads();
    ny = nyn;
    p = pn;
  }
  // Z = Y >> (pf - (e - LD))  ~ 2^e / D
  const int nz = nl + 3;
  wg_shift_right(Y, ny, pf - (e - LD), Z, nz);
  // R = 2^e - Z D, exact, over nR limbs.  Z is within a few units of 2^e / D,
  // so |R| < 2^(32 nd + 3): R is Z D's low nd + 2 limbs negated (e reaches
  // 32 (nd + 2)), and only those limbs of the product are formed
  const int nR = e >= 32L * (nd + 2) ? nd + 2 : (int)(e / 32) + 3;
  pv_mul(Z, nz, D, nd, T, nR, colbuf, cap);
  wg_sub_from_pow2(e, T, nR, T, nR, rip);
  // T2 = D zero-extended to nR (and zero up to NB for the comparison below)
  for (int j = threadIdx.x; j < (nR > NB ? nR : NB); j += blockDim.x) T2[j] = j < nd ? D[j] : 0u;
  __syncthreads();
  int guard = 0;
  while (true) {
    const bool rneg = (T[nR - 1] >> 31) != 0;
    const int cmp = rneg ? 0 : w_cmp(T, T2, nR);
    __syncthreads();
    if (rneg) {
      wg_add_i32(Z, nz, -1, rip);
      wg_add(T, nR, T2, nR, T, nR, rip);
    } else if (cmp >= 0) {
      wg_add_i32(Z, nz, 1, rip);
      wg_sub(T, T2, T, nR, rip);
    } else {
      break;
    }
    if (++guard > 16) {
      res.ok = 0;
      break;
    }
  }
  // omega = Z + [2R >= D], then the near-tie decision by the whole pivot
  wg_shift_right(T, nR, -1, Yn, nR > NB ? NB : nR);  // 2R fits: R < D < 2^(P+64)
  bool up = w_cmp(Yn, T2, nd + 1) >= 0;
  __syncthreads();
  if (up && m > 0) {
    u32* Dt = dq;  // 2 R~ - d~ (non-negative), nd + 1 limbs
    wg_sub(Yn, T2, Dt, nd + 1, rip);
    // bitlen(2R~ - d~) >= bitlen(d~) - 55 puts q~ at least 2^-56 above the
    // half-integer: no decision by delta is needed
    if (w_bitlen(Dt, nd + 1) <= LD - 56) {
      const int nm = (int)((m + 31) / 32);  // delta = d mod 2^m, nm <= nl limbs
      for (int j = threadIdx.x; j < nm; j += blockDim.x) {
        u32 v = d[j];
        if (j == nm - 1 && (m & 31)) v &= (1u << (m & 31)) - 1u;
        Yn[j] = v;
      }
      wg_shift_right(Z, nz, -1, Y, nz + 1);  // 2Z, then + 1
      if (threadIdx.x == 0) Y[0] |= 1u;
      __syncthreads();
      // X = (2Z + 1) delta over T..T2 (4 NB limbs); (2R~ - d~) 2^m beside it
      const int nX = nz + 1 + nm;
      pv_mul(Y, nz + 1, Yn, nm, T, nX, colbuf, cap);
      wg_shift_right(Dt, nd + 1, -m, colbuf, nX);
      const int c = w_cmp(T, colbuf, nX);
      __syncthreads();
      if (c > 0) up = false;
    }
  }
  if (up) wg_add_i32(Z, nz, 1, rip);
  for (int j = threadIdx.x; j < n_omega; j += blockDim.x) omega[j] = j < nz ? Z[j] : 0u;
  __syncthreads();
  return res;
}

// One wave: pivot i of the trailing matrix.
constexpr int PIVOT_THREADS = 1024;

__device__ void pivot_body(const PivotArgs& a) {
  u32* __restrict__ A = a.A;
  const Dims dm = a.dm;
  const int i = a.i;
  u32* __restrict__ d_out = a.d_out;
  i32* __restrict__ h_out = a.h_out;
  u32* __restrict__ omega_tab = a.omega;
  const int omega_stride = a.ostride;
  DevStatus* st = a.st;
  if (has_error(st)) return;
  extern __shared__ u32 lds[];
  const int nw = dm.nw, nl = dm.nl;
  u32* dl = lds + 15 * (nl + 8);
  const u32* src = A + tri_tile_index(i >> 5, i >> 5) * tile_words(nw);
  for (int l = threadIdx.x; l < nw; l += blockDim.x) dl[l] = src[in_tile(i, i, l)];
  __syncthreads();
  if (a.from_row) {
    // u = rnd(a_(i,j) / 2^h_j), b = rnd(u w_j / 2^P) for j = i - 1, the same
    // steps as the column step of column j for row i (col_body), then
    // a_ii - b u = a_ii - |b| |u| (b is zero or has the sign of u)
    const int NB = nl + 8, j = i - 1;
    u32* As = lds;              // a_ij, nw limbs
    u32* Us = lds + 2 * NB;     // |u|, nl + 1 limbs
    u32* Ws = lds + 3 * NB;     // w_j
    u32* Pr = lds + 4 * NB;     // |u| w_j + 2^(P-1), 2 nl + 1 limbs
    u32* Pt = lds + 6 * NB;     // |b| |u|, nw limbs
    int* flag = (int*)(lds + 8 * NB);
    u32* buf = lds + 9 * NB;    // 6 NB: product scratch and carry chains
    const size_t cap = (size_t)6 * NB * 4;
    const u32 lim_top = 0x60000000u;  // 3 * 2^(P-3) in the top limb
    const u32* srcj = A + tri_tile_index(i >> 5, j >> 5) * tile_words(nw);
    for (int l = threadIdx.x; l < nw; l += blockDim.x) As[l] = srcj[in_tile(i, j, l)];
    const u32* om = omega_tab + (size_t)j * omega_stride;
    for (int l = threadIdx.x; l < nl + 4; l += blockDim.x) Ws[l] = l < omega_stride ? om[l] : 0u;
    __syncthreads();
    if (wave_id() == 0) {
      const bool nega = (As[nw - 1] >> 31) != 0;
      if (nega) w_neg(As, nw);
      wsync();
      const int hj = h_out[j];
      if (hj > 0) w_add_word(As, nw, (hj - 1) >> 5, 1u << ((hj - 1) & 31));
      wsync();
      w_shift_right(As, nw, hj, Us, nl + 1);
      wsync();
      if (lane_id() == 0) flag[0] = (Us[nl] != 0 || Us[nl - 1] >= lim_top) ? 1 : 0;
    }
    __syncthreads();
    // an overflow is reported by the column step of column j, which sees the
    // same row: this pivot leaves everything as it is
    if (flag[0]) return;
    pv_mul(Us, nl, Ws, nl + 1, Pr, 2 * nl + 1, buf, cap);
    if (wave_id() == 0) {
      w_add_word(Pr, 2 * nl + 1, nl - 1, 0x80000000u);
      wsync();
      if (lane_id() == 0) flag[1] = (Pr[2 * nl] != 0 || Pr[2 * nl - 1] >= lim_top) ? 1 : 0;
    }
    __syncthreads();
    if (flag[1]) return;
    pv_mul(Pr + nl, nl, Us, nl, Pt, nw, buf, cap);
    wg_sub(dl, Pt, dl, nw, buf);
  } else if (a.sub_b) {
    // a_ii - b u, exact: |b| |u| by the workgroup product, then subtracted or
    // added by the signs (the scratch regions of the reciprocal are free here)
    const int NB = nl + 8;
    u32* Bs = lds;            // |b|
    u32* Us = lds + NB;       // |u|
    u32* Pt = lds + 2 * NB;   // |b u| (2 NB)
    u32* buf = lds + 9 * NB;  // 6 NB: product scratch and carry chains
    for (int l = threadIdx.x; l < NB; l += blockDim.x) {
      Bs[l] = l < nl ? a.sub_b[l] : 0u;
      Us[l] = l < nl ? a.sub_u[l] : 0u;
    }
    __syncthreads();
    const bool nb = (Bs[nl - 1] >> 31) != 0, nu = (Us[nl - 1] >> 31) != 0;
    __syncthreads();
    if (nb) wg_neg(Bs, nl, buf);
    if (nu) wg_neg(Us, nl, buf);
    pv_mul(Bs, nl, Us, nl, Pt, nw, buf, (size_t)6 * NB * 4);
    if (nb == nu) {
      wg_sub(dl, Pt, dl, nw, buf);
    } else {
      wg_add(dl, nw, Pt, nw, dl, nw, buf);
    }
  }
  const bool neg = (dl[nw - 1] >> 31) != 0;
  if (neg || w_is_zero(dl, nw)) {
    if (threadIdx.x == 0) set_status(st, HL_ENOTPD, i);
    return;
  }
  for (int l = threadIdx.x; l < nw; l += blockDim.x) d_out[(size_t)i * nw + l] = dl[l];
  PivotOut po = pivot_recip(dl, nw, dm.P, omega_tab + (size_t)i * omega_stride, omega_stride, lds, nl);
  if (threadIdx.x == 0) {
    h_out[i] = po.h;
    if (!po.ok) set_status(st, HL_ENOCONV, i);
  }
}

__global__ __launch_bounds__(PIVOT_THREADS) void k_pivot(PivotArgs a) { pivot_body(a); }

// one workgroup per instance of a batch
__global__ __launch_bounds__(PIVOT_THREADS) void k_pivot_b(const PivotArgs* __restrict__ tab) {
  pivot_body(tab[blockIdx.x]);
}

// ---------------------------------------------------------------------------
// Factor columns of pivot i for rows r in [r0, NT):
//   u_r = rnd(a_ri / 2^h_i),  b_r = rnd(u_r w_i / 2^P),
// both two's complement over nl limbs; rows r <= i and r >= N give zeros.
// u goes to the panel buffer, b to the multiplier array L (column i).  One
// workgroup of COL_THREADS per row: the product u w is formed by all its waves.
constexpr int COL_THREADS = 256;

// mcap > 0: the product u w by the one-workgroup int8 MFMA product (pv_mul),
// its scratch of mcap bytes at cb; 0: the product scan on the vector ALU
__device__ void col_body(const ColArgs& a, int bx, size_t mcap = 0) {
  const u32* __restrict__ A = a.A;
  const Dims dm = a.dm;
  const int i = a.i;
  const i32* __restrict__ h_tab = a.h;
  const u32* __restrict__ omega_tab = a.omega;
  const int omega_stride = a.ostride;
  DevStatus* st = a.st;
  if (has_error(st)) return;
  const int r = a.r0 + bx;
  if (r >= dm.NT) return;
  u32* __restrict__ u_out = a.u_out;
  u32* __restrict__ l_col = a.l_col;
  const int nl = dm.nl, nw = dm.nw;
  u32* uo = u_out + (size_t)r * nl;
  u32* bo = l_col + (size_t)r * nl;
  if (r <= i || r >= dm.N) {
    for (int l = threadIdx.x; l < nl; l += blockDim.x) {
      uo[l] = 0;
      bo[l] = 0;
    }
    return;
  }
  extern __shared__ u32 lds[];
  int* flag = (int*)lds;              // 4
  u32* As = lds + 4;                  // nw + 4
  u32* Us = As + nw + 4;              // nl + 4
  u32* Ws = Us + nl + 4;              // nl + 4
  u32* Pr = Ws + nl + 4;              // 2 nl + 4
  u32* cb = Pr + 2 * nl + 4;          // 3 (2 nl + 1)
  const int w0 = wave_id() == 0;
  const u32* src = A + tri_tile_index(r >> 5, i >> 5) * tile_words(nw);
  for (int l = threadIdx.x; l < nw; l += blockDim.x) As[l] = src[in_tile(r, i, l)];
  const u32* om = omega_tab + (size_t)i * omega_stride;
  for (int l = threadIdx.x; l < nl + 4; l += blockDim.x) Ws[l] = l < omega_stride ? om[l] : 0u;
  __syncthreads();
  const bool neg = (As[nw - 1] >> 31) != 0;
  const u32 lim_top = 0x60000000u;  // 3 * 2^(P-3) in the top limb
  if (w0) {
    if (neg) w_neg(As, nw);
    wsync();
    const int h = h_tab[i];
    if (h > 0) w_add_word(As, nw, (h - 1) >> 5, 1u << ((h - 1) & 31));
    wsync();
    w_shift_right(As, nw, h, Us, nl + 1);
    wsync();
    if (lane_id() == 0) flag[0] = (Us[nl] != 0 || Us[nl - 1] >= lim_top) ? 1 : 0;
  }
  __syncthreads();
  if (flag[0]) {
    if (threadIdx.x == 0) set_status(st, HL_EOVERFLOW, i);
    return;
  }
  // b = (u w + 2^(P-1)) >> P: limbs nl .. 2nl of the product plus the half
  if (mcap)
    pv_mul(Us, nl, Ws, nl + 1, Pr, 2 * nl + 1, cb, mcap);
  else
    g_mul(Us, nl, Ws, nl + 1, Pr, 2 * nl + 1, cb);
  if (w0) {
    w_add_word(Pr, 2 * nl + 1, nl - 1, 0x80000000u);
    wsync();
    if (lane_id() == 0) flag[1] = (Pr[2 * nl] != 0 || Pr[2 * nl - 1] >= lim_top) ? 1 : 0;
    wsync();
    if (!flag[1]) {
      if (neg) {
        w_neg(Us, nl);
        w_neg(Pr + nl, nl);
      }
      wsync();
      for (int l = lane_id(); l < nl; l += WAVE) {
        uo[l] = Us[l];
        bo[l] = Pr[nl + l];
      }
    }
  }
  __syncthreads();
  if (flag[1] && threadIdx.x == 0) set_status(st, HL_EOVERFLOW, i);
}

__global__ __launch_bounds__(COL_THREADS) void k_col(ColArgs a) { col_body(a, blockIdx.x); }

// batch: blockIdx.y is the instance, blockIdx.x the row offset
__global__ __launch_bounds__(COL_THREADS) void k_col_b(const ColArgs* __restrict__ tab) {
  col_body(tab[blockIdx.y], blockIdx.x);
}

// The MFMA form's column step in one launch: one workgroup per row, the
// product u w by the workgroup's int8 MFMAs (same bits as k_col).
constexpr int COL_M_THREADS = 1024;
__global__ __launch_bounds__(COL_M_THREADS) void k_col_m(ColArgs a, size_t mcap) { col_body(a, blockIdx.x, mcap); }

// ---------------------------------------------------------------------------
// Exact update of few entries, A[r][c] -= sum_i b_ri u_ci (UpdArgs), one
// workgroup per entry (blockIdx.x = (r - r_lo) (c_hi - c_lo) + c - c_lo): each
// product |b| |u| by the workgroup's int8 MFMAs, then subtracted or added by
// the signs, modulo 2^(32 nw) as every form of the update.  For launches whose
// entries are too few to fill the Toeplitz-form kernel's work items.
constexpr int UPD_WG_THREADS = 1024;
__global__ __launch_bounds__(UPD_WG_THREADS) void k_upd_wg(UpdArgs g, size_t mcap) {
  const int ncols = g.c_hi - g.c_lo;
  const int r = g.r_lo + (int)(blockIdx.x / ncols), c = g.c_lo + (int)(blockIdx.x % ncols);
  if (r >= g.r_hi || (g.tri && r < c)) return;
  if (has_error(g.st)) return;
  const int nl = g.nl, nw = g.nw, NB = nl + 8;
  const size_t tix = g.tri ? tri_tile_index(r >> 5, c >> 5) : (size_t)(r >> 5) * g.ntc + (c >> 5);
  u32* At = g.A + tix * tile_words(nw);
  extern __shared__ u32 lds[];
  u32* Bs = lds;              // |b|
  u32* Us = Bs + NB;          // |u|
  u32* Pt = Us + NB;          // |b u|, nw + 8
  u32* Es = Pt + nw + 8;      // the entry, nw + 8
  u32* buf = Es + nw + 8;     // mcap bytes: product scratch and carry chains
  for (int l = threadIdx.x; l < nw; l += blockDim.x) Es[l] = At[in_tile(r, c, l)];
  const size_t rsb = g.rsb ? g.rsb : (size_t)nl;
  for (int il = 0; il < g.npan; ++il) {
    const u32* b = g.Bop + il * g.ldb + (size_t)r * rsb;
    const u32* u = g.Uop + il * g.ldu + (size_t)c * nl;
    for (int l = threadIdx.x; l < NB; l += blockDim.x) {
      Bs[l] = l < nl ? b[l] : 0u;
      Us[l] = l < nl ? u[l] : 0u;
    }
    __syncthreads();
    const bool nb = (Bs[nl - 1] >> 31) != 0, nu = (Us[nl - 1] >> 31) != 0;
    __syncthreads();
    if (nb) wg_neg(Bs, nl, buf);
    if (nu) wg_neg(Us, nl, buf);
    pv_mul(Bs, nl, Us, nl, Pt, nw, buf, mcap);
    if (nb == nu) {
      wg_sub(Es, Pt, Es, nw, buf);
    } else {
      wg_add(Es, nw, Pt, nw, Es, nw, buf);
    }
  }
  for (int l = threadIdx.x; l < nw; l += blockDim.x) At[in_tile(r, c, l)] = Es[l];
}

// ---------------------------------------------------------------------------
// The same column in three launches, for the MFMA form: k_col_u forms the
// signed u_r, the product P_r = u_r w_i runs as an int8 MFMA GEMM (Toeplitz
// form, all rows against the one w_i), and k_col_fin rounds
// b_r = sign(P_r) ((|P_r| + 2^(P-1)) >> P).  Same bits as k_col.  One wave per row.
__device__ __forceinline__ void col_u_body(const ColArgs& a, int bx) {
  const Dims dm = a.dm;
  const int i = a.i, r = a.r0 + bx;
  DevStatus* st = a.st;
  if (has_error(st) || r >= dm.NT) return;
  const int nl = dm.nl, nw = dm.nw;
  u32* uo = a.u_out + (size_t)r * nl;
  if (r <= i || r >= dm.N) {
    for (int l = lane_id(); l < nl; l += WAVE) uo[l] = 0;
    return;
  }
  extern __shared__ u32 lds[];
  u32* As = lds;            // nw
  u32* Us = As + nw;        // nl + 1
  const u32* src = a.A + tri_tile_index(r >> 5, i >> 5) * tile_words(nw);
  for (int l = lane_id(); l < nw; l += WAVE) As[l] = src[in_tile(r, i, l)];
  wsync();
  const bool neg = (As[nw - 1] >> 31) != 0;
  if (neg) w_neg(As, nw);
  wsync();
  const int h = a.h[i];
  if (h > 0) w_add_word(As, nw, (h - 1) >> 5, 1u << ((h - 1) & 31));
  wsync();
  w_shift_right(As, nw, h, Us, nl + 1);
  wsync();
  if (Us[nl] != 0 || Us[nl - 1] >= 0x60000000u) {  // |u| < 3 2^(P-3)
    if (lane_id() == 0) set_status(st, HL_EOVERFLOW, i);
    return;
  }
  if (neg) w_neg(Us, nl);
  wsync();
  for (int l = lane_id(); l < nl; l += WAVE) uo[l] = Us[l];
}

__global__ __launch_bounds__(64) void k_col_u(ColArgs a) { col_u_body(a, blockIdx.x); }

// batch: blockIdx.y is the instance
__global__ __launch_bounds__(64) void k_col_u_b(const ColArgs* __restrict__ tab) { col_u_body(tab[blockIdx.y], blockIdx.x); }

// P: row r at P + r ldp (ldp >= 2 nl + 1 limbs, two's complement)
__device__ __forceinline__ void col_fin_body(const ColArgs& a, const u32* __restrict__ P, int ldp, int bx) {
  const Dims dm = a.dm;
  const int i = a.i, r = a.r0 + bx;
  DevStatus* st = a.st;
  if (has_error(st) || r >= dm.NT) return;
  const int nl = dm.nl;
  u32* bo = a.l_col + (size_t)r * nl;
  if (r <= i || r >= dm.N) {
    for (int l = lane_id(); l < nl; l += WAVE) bo[l] = 0;
    return;
  }
  extern __shared__ u32 lds[];
  u32* Ps = lds;  // ldp
  for (int l = lane_id(); l < ldp; l += WAVE) Ps[l] = P[(size_t)r * ldp + l];
  wsync();
  const bool neg = (Ps[ldp - 1] >> 31) != 0;
  if (neg) w_neg(Ps, ldp);
  wsync();
  w_add_word(Ps, ldp, nl - 1, 0x80000000u);
  wsync();
  bool over = Ps[2 * nl - 1] >= 0x60000000u;
  for (int l = 2 * nl; l < ldp; ++l) over = over || Ps[l] != 0;
  if (over) {
    if (lane_id() == 0) set_status(st, HL_EOVERFLOW, i);
    return;
  }
  if (neg) w_neg(Ps + nl, nl);
  wsync();
  for (int l = lane_id(); l < nl; l += WAVE) bo[l] = Ps[nl + l];
}

__global__ __launch_bounds__(64) void k_col_fin(ColArgs a, const u32* __restrict__ P, int ldp) {
  col_fin_body(a, P, ldp, blockIdx.x);
}

__global__ __launch_bounds__(64) void k_col_fin_b(const ColFinArgs* __restrict__ tab) {
  const ColFinArgs& f = tab[blockIdx.y];
  col_fin_body(f.c, f.P, f.ldp, blockIdx.x);
}

// ---------------------------------------------------------------------------
__global__ void k_fill_u32(u32* __restrict__ p, size_t n, u32 v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
// test hooks
__global__ __launch_bounds__(64) void k_debug_mul(const u32* a, int na, const u32* b, int nb, u32* out,
                                                  int nout) {
  w_mul(a, na, b, nb, out, nout);
}

// the one-workgroup MFMA product, on operands staged in LDS
__global__ __launch_bounds__(1024) void k_debug_mul_wg(const u32* a, int na, const u32* b, int nb, u32* out,
                                                     int nout) {
  extern __shared__ u32 lds[];
  u32* as = lds;
  u32* bs = as + ((na + 3) & ~3);
  u32* os = bs + ((nb + 3) & ~3);
  u32* sc = os + ((nout + 3) & ~3);
  for (int i = threadIdx.x; i < na; i += blockDim.x) as[i] = a[i];
  for (int i = threadIdx.x; i < nb; i += blockDim.x) bs[i] = b[i];
  __syncthreads();
  wg_mfma_mul(as, na, bs, nb, os, nout, sc);
  for (int i = threadIdx.x; i < nout; i += blockDim.x) out[i] = os[i];
}

__global__ __launch_bounds__(PIVOT_THREADS) void k_debug_recip(const u32* d, int nd, int P, int nl, u32* omega,
                                                               int n_omega, i32* h) {
  extern __shared__ u32 lds[];
  u32* dl = lds + 15 * (nl + 8);
  for (int l = threadIdx.x; l < 2 * nl; l += blockDim.x) dl[l] = l < nd ? d[l] : 0u;
  __syncthreads();
  PivotOut po = pivot_recip(dl, 2 * nl, P, omega, n_omega, lds, nl);
  if (threadIdx.x == 0) h[0] = po.ok ? po.h : -1;
}

// ---------------------------------------------------------------------------
// host launchers
size_t pivot_lds_bytes(int nl) { return (size_t)(15 * (nl + 8) + 2 * nl + 8) * 4; }
size_t col_lds_bytes(int nl) { return (size_t)(4 + 2 * nl + 4 + 2 * (nl + 4) + 2 * nl + 4 + 3 * (2 * nl + 1)) * 4; }

hipError_t launch_scales(const u32* mu, const i64* mu_exp, int w, int N, int E, i32* s, DevStatus* st,
                         hipStream_t stream) {
  const int nJ = (N + E - 1) / E;
  hipLaunchKernelGGL(k_scales, dim3((nJ + 255) / 256), dim3(256), 0, stream, mu, mu_exp, w, N, E, s, st);
  return hipGetLastError();
}

hipError_t launch_load(const u32* mu, const i64* mu_exp, int w, const i32* s, const Dims& dm, u32* A,
                       DevStatus* st, hipStream_t stream) {
  const size_t ntiles = (size_t)dm.nt * (dm.nt + 1) / 2;
  hipLaunchKernelGGL(k_load, dim3((unsigned)ntiles), dim3(1024), 0, stream, mu, mu_exp, w, s, dm, A, st);
  return hipGetLastError();
}

// kernels that may need more than 64 KiB of dynamic LDS (up to the 160 KiB of a CU)
static hipError_t allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_pivot(u32* A, const Dims& dm, int i, u32* d_out, i32* h_out, u32* omega, int ostride,
                        DevStatus* st, hipStream_t stream, const u32* sub_b, const u32* sub_u, int from_row) {
  hipError_t e = allow_lds((const void*)k_pivot, pivot_lds_bytes(dm.nl));
  if (e != hipSuccess) return e;
  if ((sub_b == nullptr) != (sub_u == nullptr)) return hipErrorInvalidValue;
  if (from_row && (sub_b || i < 1)) return hipErrorInvalidValue;
  const PivotArgs a{A, dm, i, d_out, h_out, omega, ostride, st, sub_b, sub_u, from_row};
  hipLaunchKernelGGL(k_pivot, dim3(1), dim3(PIVOT_THREADS), pivot_lds_bytes(dm.nl), stream, a);
  return hipGetLastError();
}

hipError_t launch_col(const u32* A, const Dims& dm, int i, int r0, const i32* h, const u32* omega,
                      int ostride, u32* u_out, u32* l_col, DevStatus* st, hipStream_t stream) {
  const int nrows = dm.NT - r0;
  if (nrows <= 0) return hipSuccess;
  const ColArgs a{A, dm, i, r0, h, omega, ostride, u_out, l_col, st};
  hipError_t e = allow_lds((const void*)k_col, col_lds_bytes(dm.nl));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col, dim3(nrows), dim3(COL_THREADS), col_lds_bytes(dm.nl), stream, a);
  return hipGetLastError();
}

hipError_t launch_upd_wg(const UpdArgs& g, hipStream_t stream) {
  if (g.r_hi <= g.r_lo || g.c_hi <= g.c_lo || g.npan <= 0) return hipSuccess;
  const int nl = g.nl;
  const size_t fixed = (size_t)(2 * (nl + 8) + 2 * (g.nw + 8)) * 4;
  size_t mcap = (size_t)3 * (2 * nl + 1) * 4;
  if (wm_scratch_bytes(nl, nl) > mcap) mcap = wm_scratch_bytes(nl, nl);
  mcap = (mcap + 15) / 16 * 16;
  if (fixed + mcap > (size_t)160 * 1024) return hipErrorInvalidValue;
  hipError_t e = allow_lds((const void*)k_upd_wg, fixed + mcap);
  if (e != hipSuccess) return e;
  const size_t entries = (size_t)(g.r_hi - g.r_lo) * (g.c_hi - g.c_lo);
  hipLaunchKernelGGL(k_upd_wg, dim3((unsigned)entries), dim3(UPD_WG_THREADS), fixed + mcap, stream, g, mcap);
  return hipGetLastError();
}

hipError_t launch_col_m(const u32* A, const Dims& dm, int i, int r0, const i32* h, const u32* omega,
                        int ostride, u32* u_out, u32* l_col, DevStatus* st, hipStream_t stream) {
  const int nrows = dm.NT - r0;
  if (nrows <= 0) return hipSuccess;
  const int nl = dm.nl;
  const size_t fixed = (size_t)(6 * nl + 20) * 4;  // flag, As, Us, Ws, Pr as in col_body
  size_t mcap = (size_t)3 * (2 * nl + 1) * 4;
  if (wm_scratch_bytes(nl, nl + 1) > mcap) mcap = wm_scratch_bytes(nl, nl + 1);
  mcap = (mcap + 15) / 16 * 16;
  if (fixed + mcap > (size_t)160 * 1024) return hipErrorInvalidValue;
  const ColArgs a{A, dm, i, r0, h, omega, ostride, u_out, l_col, st};
  hipError_t e = allow_lds((const void*)k_col_m, fixed + mcap);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_m, dim3(nrows), dim3(COL_M_THREADS), fixed + mcap, stream, a, mcap);
  return hipGetLastError();
}

hipError_t launch_col_u(const u32* A, const Dims& dm, int i, int r0, const i32* h, u32* u_out, DevStatus* st,
                        hipStream_t stream) {
  const int nrows = dm.NT - r0;
  if (nrows <= 0) return hipSuccess;
  const ColArgs a{A, dm, i, r0, h, nullptr, 0, u_out, nullptr, st};
  const size_t lds = (size_t)(dm.nw + dm.nl + 1) * 4;
  hipError_t e = allow_lds((const void*)k_col_u, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_u, dim3(nrows), dim3(64), lds, stream, a);
  return hipGetLastError();
}

hipError_t launch_col_fin(const Dims& dm, int i, int r0, const u32* P, int ldp, u32* l_col, DevStatus* st,
                          hipStream_t stream) {
  const int nrows = dm.NT - r0;
  if (nrows <= 0) return hipSuccess;
  if (ldp < 2 * dm.nl + 1) return hipErrorInvalidValue;
  const ColArgs a{nullptr, dm, i, r0, nullptr, nullptr, 0, nullptr, l_col, st};
  const size_t lds = (size_t)ldp * 4;
  hipError_t e = allow_lds((const void*)k_col_fin, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_fin, dim3(nrows), dim3(64), lds, stream, a, P, ldp);
  return hipGetLastError();
}

hipError_t launch_col_u_batch(const ColArgs* tab, int count, int rows_max, int nl_max, hipStream_t stream) {
  if (count <= 0 || rows_max <= 0) return hipSuccess;
  const size_t lds = (size_t)(3 * nl_max + 1) * 4;  // nw + nl + 1 words
  hipError_t e = allow_lds((const void*)k_col_u_b, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_u_b, dim3(rows_max, count), dim3(64), lds, stream, tab);
  return hipGetLastError();
}

hipError_t launch_col_fin_batch(const ColFinArgs* tab, int count, int rows_max, int ldp_max, hipStream_t stream) {
  if (count <= 0 || rows_max <= 0) return hipSuccess;
  const size_t lds = (size_t)ldp_max * 4;
  hipError_t e = allow_lds((const void*)k_col_fin_b, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_fin_b, dim3(rows_max, count), dim3(64), lds, stream, tab);
  return hipGetLastError();
}

hipError_t launch_pivot_batch(const PivotArgs* tab, int count, int nl_max, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipError_t e = allow_lds((const void*)k_pivot_b, pivot_lds_bytes(nl_max));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pivot_b, dim3(count), dim3(PIVOT_THREADS), pivot_lds_bytes(nl_max), stream, tab);
  return hipGetLastError();
}

hipError_t launch_col_batch(const ColArgs* tab, int count, int rows_max, int nl_max, hipStream_t stream) {
  if (count <= 0 || rows_max <= 0) return hipSuccess;
  hipError_t e = allow_lds((const void*)k_col_b, col_lds_bytes(nl_max));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_b, dim3(rows_max, count), dim3(COL_THREADS), col_lds_bytes(nl_max), stream, tab);
  return hipGetLastError();
}

hipError_t launch_fill(u32* p, size_t n, u32 v, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_debug_mul(const u32* a, int na, const u32* b, int nb, u32* out, int nout,
                            hipStream_t stream) {
  hipLaunchKernelGGL(k_debug_mul, dim3(1), dim3(64), 0, stream, a, na, b, nb, out, nout);
  return hipGetLastError();
}

hipError_t launch_debug_mul_wg(const u32* a, int na, const u32* b, int nb, u32* out, int nout, int threads,
                               hipStream_t stream) {
  if (threads != 256 && threads != 1024) return hipErrorInvalidValue;
  const size_t lds = (size_t)(((na + 3) & ~3) + ((nb + 3) & ~3) + ((nout + 3) & ~3)) * 4 + wm_scratch_bytes(na, nb);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = allow_lds((const void*)k_debug_mul_wg, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_debug_mul_wg, dim3(1), dim3(threads), lds, stream, a, na, b, nb, out, nout);
  return hipGetLastError();
}

hipError_t launch_debug_recip(const u32* d, int nd, int P, u32* omega, int n_omega, i32* h,
                              hipStream_t stream) {
  const int nl = P / 32;
  hipError_t e = allow_lds((const void*)k_debug_recip, pivot_lds_bytes(nl));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_debug_recip, dim3(1), dim3(PIVOT_THREADS), pivot_lds_bytes(nl), stream, d, nd, P, nl, omega,
                     n_omega, h);
  return hipGetLastError();
}

}  // namespace hl
