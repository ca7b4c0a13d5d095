// Eigen-step: lambda_1 ~= 1 / lambda_max of the k x k block of H^-1 (Section 4.2),
// and the same for the leading (k-1) x (k-1) block (truncation estimate,
// Section 4.5).  The paper casts the block to double and calls a library
// eigen-solver; here it stays in multiprecision and no FP64 arithmetic is used.
//
// Arithmetic: multiprecision floating point (sign, exponent, mantissa of up to
// NWM 32-bit limbs normalised to [1/2, 1)), built on the exact multi-limb
// primitives; a working precision of nw limbs uses only the top nw limbs.
//
// Iteration (one workgroup per block): shifted inverse iteration with Rayleigh
// quotients inside a bracket lo <= lambda_max < hi.
//   * every Rayleigh quotient y'By / y'y is a lower bound of lambda_max;
//   * a shift sigma with sigma I - B positive definite (all LDL^T pivots > 0)
//     is an upper bound; a trial shift that fails the test is a lower bound;
//   * the upper bound starts at Gershgorin's bound; each step solves
//     (hi I - B) z = y, normalises z by a power of two, takes its Rayleigh
//     quotient, and tries hi' = lo + c (hi - lo)^2 / hi, the size the error of
//     the Rayleigh quotient would have after one step of the iteration;
//   * the working precision grows with the number of bits the bracket has
//     resolved, so only the last steps run at full precision.
// The iteration stops when the bracket is narrower than 2^-(P+32) relative.
#include <thread>

#include "hl_kernels.hpp"
#include "mp_mfma.hpp"
#include "hl_host.hpp"

namespace hl {

constexpr int EIG_WAVES = 8;
constexpr int EIG_THREADS = EIG_WAVES * WAVE;
constexpr int EIG_MAXIT = 400;
constexpr int EIG_NSCAL = 24;
// matrices of the workspace: 0 the k x k block, 1 its leading (k-1) x (k-1)
// block; 2 j and 2 j + 1 (j = 1, 2) the same less the eigenpairs found in
// matrices 2 j - 2 and 2 j - 1 (deflation, for the next eigenvalues)
constexpr int EIG_MATS = 6;
// flag words at the head of the workspace: 8 per matrix for matrices 0 and 1,
// the iteration trace of those two at 16 .. 63, 8 per matrix for the rest from 64
constexpr int EIG_FLAG_INTS = 64 + 8 * (EIG_MATS - 2);
__host__ __device__ __forceinline__ int eig_flag_off(int which) { return which < 2 ? 8 * which : 64 + 8 * (which - 2); }

// ---------------------------------------------------------------------------
// multiprecision floats in global memory: header (sign, exp) + NWM limbs
struct FpRef {
  int* hdr;  // hdr[0] = sign (0/1), hdr[1] = exponent; zero when hdr[0] == 2
  u32* m;    // NWM limbs, significant limbs at the top
};

struct FpCtx {
  int NWM;   // limb capacity
  int nw;    // working precision in limbs (<= NWM - 1)
  u32* la;   // per-wave LDS scratch, 2 * (NWM + 4) words
  u32* lb;
};

constexpr int FPZERO_TAG = 2;

__device__ __forceinline__ bool fp_is_zero(const FpRef& x) { return x.hdr[0] == FPZERO_TAG; }

__device__ void fp_set_zero(const FpCtx& c, FpRef z) {
  for (int j = lane_id(); j < c.NWM; j += WAVE) z.m[j] = 0;
  if (lane_id() == 0) {
    z.hdr[0] = FPZERO_TAG;
    z.hdr[1] = 0;
  }
  wsync();
}

__device__ void fp_copy(const FpCtx& c, FpRef z, const FpRef& x) {
  const int s0 = x.hdr[0], s1 = x.hdr[1];
  for (int j = lane_id(); j < c.NWM; j += WAVE) z.m[j] = x.m[j];
  if (lane_id() == 0) {
    z.hdr[0] = s0;
    z.hdr[1] = s1;
  }
  wsync();
}

// z = value of the signed integer (two's complement, n limbs) at src
__device__ void fp_from_int(const FpCtx& c, FpRef z, const u32* src, int n) {
  u32* t = c.la;
  for (int j = lane_id(); j < n; j += WAVE) t[j] = src[j];
  wsync();
  const bool neg = (t[n - 1] >> 31) != 0;
  if (neg) w_neg(t, n);
  wsync();
  const int bl = w_bitlen(t, n);
  if (bl == 0) {
    fp_set_zero(c, z);
    return;
  }
  // mantissa = t << (32 NWM - bl): its top bit lands on bit 32 NWM - 1
  const long sh = 32L * c.NWM - bl;
  for (int j = lane_id(); j < c.NWM; j += WAVE) {
    u32 v = sh >= 0 ? limb_shl(t, n, sh, j) : limb_shr(t, n, -sh, j);
    if (j < c.NWM - c.nw) v = 0;
    z.m[j] = v;
  }
  if (lane_id() == 0) {
    z.hdr[0] = neg ? 1 : 0;
    z.hdr[1] = bl;  // value = (M / 2^(32 NWM)) 2^bl
  }
  wsync();
}

// z = x * y at working precision (z may alias x or y)
__device__ void fp_mul(const FpCtx& c, FpRef z, const FpRef& x, const FpRef& y) {
  if (fp_is_zero(x) || fp_is_zero(y)) {
    fp_set_zero(c, z);
    return;
  }
  const int nw = c.nw, top = c.NWM - nw;
  u32* A = c.la;
  u32* B = c.lb;
  for (int j = lane_id(); j < nw; j += WAVE) {
    A[j] = x.m[top + j];
    B[j] = y.m[top + j];
  }
  const int sx = x.hdr[0], sy = y.hdr[0], e = x.hdr[1] + y.hdr[1];
  wsync();
  // limbs nw-1 .. 2nw-1 of A*B land on z.m[top-1 .. NWM)
  const int nch = (2 * nw + WAVE - 1) / WAVE;
  u32* zm = z.m;
  w_mul_stream(A, nw, B, nw, nch, [&](int ch, u32 limb) {
    const int p = ch * WAVE + lane_id();
    if (p >= nw - 1 && p < 2 * nw) zm[top - 1 + (p - (nw - 1))] = limb;
  });
  wsync();
  const bool low = (zm[c.NWM - 1] >> 31) == 0;
  if (low) {
    // shift z.m[top-1 .. NWM) left by one bit through LDS
    for (int j = top - 1 + lane_id(); j < c.NWM; j += WAVE) A[j - (top - 1)] = zm[j];
    wsync();
    for (int j = top + lane_id(); j < c.NWM; j += WAVE)
      zm[j] = (A[j - (top - 1)] << 1) | (A[j - top] >> 31);
  }
  wsync();
  for (int j = lane_id(); j < top; j += WAVE) zm[j] = 0;
  if (lane_id() == 0) {
    z.hdr[0] = sx ^ sy;
    z.hdr[1] = e - (low ? 1 : 0);
  }
  wsync();
}

// z = x + (neg_y ? -y : y) at working precision (z may alias x or y)
__device__ void fp_add(const FpCtx& c, FpRef z, const FpRef& x0, const FpRef& y0, bool neg_y) {
  const int nw = c.nw, top = c.NWM - nw;
  const bool xz = fp_is_zero(x0), yz = fp_is_zero(y0);
  if (yz) {
    if (z.m != x0.m) fp_copy(c, z, x0);
    wsync();
    return;
  }
  if (xz) {
    if (z.m != y0.m) fp_copy(c, z, y0);
    wsync();
    if (neg_y && lane_id() == 0) z.hdr[0] ^= 1;
    wsync();
    return;
  }
  int sx = x0.hdr[0], sy = y0.hdr[0] ^ (neg_y ? 1 : 0);
  int ex = x0.hdr[1], ey = y0.hdr[1];
  const FpRef* X = &x0;
  const FpRef* Y = &y0;
  if (ey > ex) {
    X = &y0;
    Y = &x0;
    int t = sx; sx = sy; sy = t;
    t = ex; ex = ey; ey = t;
  }
  const long d = (long)ex - ey;
  const int n = nw + 3;  // 2 guard limbs below, 1 carry limb above
  u32* A = c.la;
  u32* B = c.lb;
  for (int j = lane_id(); j < n; j += WAVE) {
    A[j] = (j >= 2 && j < nw + 2) ? X->m[top + j - 2] : 0u;
  }
  // B = (Y limbs placed like A) >> d
  for (int j = lane_id(); j < n; j += WAVE) {
    const long src = (long)j + (d >> 5) - 2;  // limb index into Y's nw significant limbs
    const int r = (int)(d & 31);
    u32 lo = (src >= 0 && src < nw) ? Y->m[top + src] : 0u;
    u32 hi = (src + 1 >= 0 && src + 1 < nw) ? Y->m[top + src + 1] : 0u;
    B[j] = (j == n - 1) ? 0u : (r ? ((lo >> r) | (hi << (32 - r))) : lo);
    if (d > 32L * (nw + 4)) B[j] = 0;
  }
  wsync();
  int sz = sx;
  if (sx == sy) {
    w_add(A, n, B, n, A, n);
  } else {
    const int cmp = w_cmp(A, B, n);
    if (cmp == 0) {
      fp_set_zero(c, z);
      wsync();
      return;
    }
    if (cmp > 0) {
      w_sub(A, B, A, n);
    } else {
      w_sub(B, A, A, n);
      sz = sy;
    }
  }
  wsync();
  // normalise: top bit of A (n limbs) to bit 32 (nw + 2) - 1, i.e. limb n-2's top
  const int bl = w_bitlen(A, n);
  const long want = 32L * (nw + 2);
  const long sh = want - bl;  // > 0: shift left
  int e = ex - (int)sh;
  // write the top nw limbs of (A << sh) to z
  for (int j = lane_id(); j < nw; j += WAVE) {
    const int dst = j + 2;
    u32 v = sh >= 0 ? limb_shl(A, n, sh, dst) : limb_shr(A, n, -sh, dst);
    B[j] = v;
  }
  wsync();
  for (int j = lane_id(); j < c.NWM; j += WAVE) z.m[j] = j >= top ? B[j - top] : 0u;
  if (lane_id() == 0) {
    z.hdr[0] = sz;
    z.hdr[1] = e;
  }
  wsync();
}

// z = 2^k x
__device__ void fp_ldexp(FpRef z, int k) {
  if (lane_id() == 0 && z.hdr[0] != FPZERO_TAG) z.hdr[1] += k;
  wsync();
}

// sign of x - y (magnitudes and signs), -1 / 0 / 1
__device__ int fp_cmp(const FpCtx& c, const FpRef& x, const FpRef& y) {
  const bool xz = fp_is_zero(x), yz = fp_is_zero(y);
  const int sx = xz ? 0 : (x.hdr[0] ? -1 : 1), sy = yz ? 0 : (y.hdr[0] ? -1 : 1);
  if (sx != sy) return sx > sy ? 1 : -1;
  if (sx == 0) return 0;
  int mag;
  if (x.hdr[1] != y.hdr[1]) {
    mag = x.hdr[1] > y.hdr[1] ? 1 : -1;
  } else {
    mag = w_cmp(x.m, y.m, c.NWM);
  }
  return sx > 0 ? mag : -mag;
}

// reciprocal by Newton's iteration y <- y + y (1 - x y) with doubling precision
__device__ void fp_recip(const FpCtx& c0, FpRef z, const FpRef& x, FpRef t1, FpRef t2) {
  FpCtx c = c0;
  // 62-bit start from the top 64 bits of the mantissa
  const u32 m1 = x.m[c.NWM - 1], m0 = x.m[c.NWM - 2];
  const u64 top = ((u64)m1 << 32) | m0;  // in [2^63, 2^64)
  const u64 top32 = top >> 32;           // [2^31, 2^32)
  u64 q = (~0ull) / (top32 + 1);  // ~ 2^32 / f, f = top32 / 2^32 in [1/2, 1)
  if (q < (1ull << 32)) q = 1ull << 32;
  // 1/x = (1 / (2f)) 2^(1 - ex), and 1 / (2f) ~ q / 2^33 in [1/2, 1)
  if (lane_id() == 0) z.hdr[0] = x.hdr[0];
  for (int j = lane_id(); j < c.NWM; j += WAVE) {
    u32 v = 0;
    // q has 33 bits; place so that bit 32 of q is bit 32 NWM - 1
    if (j == c.NWM - 1) v = (u32)(q >> 1);
    if (j == c.NWM - 2) v = (u32)(q << 31);
    z.m[j] = v;
  }
  if (lane_id() == 0) z.hdr[1] = 1 - x.hdr[1];
  wsync();
  // z ~ 1/x to ~30 bits; iterate
  const int target = c0.nw;
  int prec = 1;
  for (int it = 0; it < 40; ++it) {
    int np = 2 * prec;
    if (np > target) np = target;
    c.nw = np + 1 <= c0.NWM - 1 ? np + 1 : c0.NWM - 1;
    if (c.nw > target) c.nw = target;
    // t1 = x z ; t2 = 1 - t1 ; t1 = z t2 ; z = z + t1
    fp_mul(c, t1, x, z);
    // t2 = 1 - t1: build 1 in t2
    for (int j = lane_id(); j < c.NWM; j += WAVE) t2.m[j] = (j == c.NWM - 1) ? 0x80000000u : 0u;
    if (lane_id() == 0) {
      t2.hdr[0] = 0;
      t2.hdr[1] = 1;
    }
    wsync();
    fp_add(c, t2, t2, t1, true);
    fp_mul(c, t1, z, t2);
    fp_add(c, z, z, t1, false);
    prec = np;
    if (np >= target) {
      if (it > 0 && np == target) {
        // one extra polish step at full precision
        fp_mul(c, t1, x, z);
        for (int j = lane_id(); j < c.NWM; j += WAVE) t2.m[j] = (j == c.NWM - 1) ? 0x80000000u : 0u;
        if (lane_id() == 0) {
          t2.hdr[0] = 0;
          t2.hdr[1] = 1;
        }
        wsync();
        fp_add(c, t2, t2, t1, true);
        fp_mul(c, t1, z, t2);
        fp_add(c, z, z, t1, false);
      }
      break;
    }
  }
}

// ---------------------------------------------------------------------------
struct EigMat {
  int n;          // order of this block (k or k-1)
  int NWM;
  int* hdr;       // headers of all numbers, 2 ints each
  u32* mant;      // mantissas, NWM each
  int* flags;     // [0] status, [1] iterations
};

// number indices inside one EigMat region
__host__ __device__ __forceinline__ int ix_B(int n, int a, int b) { return a * n + b; }
__host__ __device__ __forceinline__ int ix_C(int n, int a, int b) { return n * n + a * n + b; }
__host__ __device__ __forceinline__ int ix_L(int n, int a, int b) { return 2 * n * n + a * n + b; }
__host__ __device__ __forceinline__ int ix_y(int n, int a) { return 3 * n * n + a; }
__host__ __device__ __forceinline__ int ix_z(int n, int a) { return 3 * n * n + n + a; }
__host__ __device__ __forceinline__ int ix_t(int n, int a) { return 3 * n * n + 2 * n + a; }
__host__ __device__ __forceinline__ int ix_inv(int n, int a) { return 3 * n * n + 3 * n + a; }
__host__ __device__ __forceinline__ int ix_s(int n, int j) { return 3 * n * n + 4 * n + j; }  // scalars
// per-wave scratch numbers: after the scalars
__host__ __device__ __forceinline__ int ix_w(int n, int w, int j) { return 3 * n * n + 4 * n + EIG_NSCAL + w * 4 + j; }
// per-target scratch numbers of the multi-workgroup form: n x n after the above
__host__ __device__ __forceinline__ int ix_T(int n, int a, int b) {
  return 3 * n * n + 4 * n + EIG_NSCAL + EIG_WAVES * 4 + a * n + b;
}
__host__ __device__ __forceinline__ int eig_numbers(int n) { return 4 * n * n + 4 * n + EIG_NSCAL + EIG_WAVES * 4; }

__device__ __forceinline__ FpRef num(const EigMat& M, int i) {
  return FpRef{M.hdr + 2 * i, M.mant + (size_t)i * M.NWM};
}

enum { S_HI = 0, S_LO, S_RQ, S_TRY, S_W, S_NUM, S_DEN, S_ONE, S_T1, S_T2, S_T3, S_RES };

// LDL^T of C = sigma I - B in place (C <- Schur complements, L, inv pivots);
// returns true if every pivot is positive.  All waves call it.
__device__ bool eig_factor(const EigMat& M, FpCtx c, const FpRef& sigma, int* flag_lds) {
  const int n = M.n, w = wave_id();
  // C = sigma I - B
  for (int idx = w; idx < n * n; idx += EIG_WAVES) {
    const int a = idx / n, b = idx % n;
    FpRef C = num(M, ix_C(n, a, b));
    FpRef B = num(M, ix_B(n, a, b));
    if (a == b) fp_add(c, C, sigma, B, true);
    else {
      fp_copy(c, C, B);
      wsync();
      if (lane_id() == 0 && C.hdr[0] != FPZERO_TAG) C.hdr[0] ^= 1;
    }
  }
  __syncthreads();
  for (int i = 0; i < n; ++i) {
    if (w == 0) {
      FpRef d = num(M, ix_C(n, i, i));
      const bool pos = !fp_is_zero(d) && d.hdr[0] == 0;
      if (lane_id() == 0) flag_lds[0] = pos ? 1 : 0;
      if (pos) fp_recip(c, num(M, ix_inv(n, i)), d, num(M, ix_w(n, 0, 0)), num(M, ix_w(n, 0, 1)));
    }
    __syncthreads();
    if (!flag_lds[0]) return false;
    for (int r = i + 1 + w; r < n; r += EIG_WAVES)
      fp_mul(c, num(M, ix_L(n, r, i)), num(M, ix_C(n, r, i)), num(M, ix_inv(n, i)));
    __syncthreads();
    const int m = n - i - 1;
    for (int idx = w; idx < m * m; idx += EIG_WAVES) {
      const int r = i + 1 + idx / m, cc = i + 1 + idx % m;
      if (r < cc) continue;
      FpRef T = num(M, ix_w(n, w, 0));
      fp_mul(c, T, num(M, ix_L(n, r, i)), num(M, ix_C(n, cc, i)));
      fp_add(c, num(M, ix_C(n, r, cc)), num(M, ix_C(n, r, cc)), T, true);
    }
    __syncthreads();
  }
  return true;
}

// z = C^-1 y with the factorisation above (C = L D L^T); y is preserved.
__device__ void eig_solve(const EigMat& M, FpCtx c) {
  const int n = M.n, w = wave_id();
  for (int a = w; a < n; a += EIG_WAVES) fp_copy(c, num(M, ix_t(n, a)), num(M, ix_y(n, a)));
  __syncthreads();
  // forward: t_r -= L_rj t_j
  for (int j = 0; j < n; ++j) {
    for (int r = j + 1 + w; r < n; r += EIG_WAVES) {
      FpRef T = num(M, ix_w(n, w, 0));
      fp_mul(c, T, num(M, ix_L(n, r, j)), num(M, ix_t(n, j)));
      fp_add(c, num(M, ix_t(n, r)), num(M, ix_t(n, r)), T, true);
    }
    __syncthreads();
  }
  for (int a = w; a < n; a += EIG_WAVES) fp_mul(c, num(M, ix_t(n, a)), num(M, ix_t(n, a)), num(M, ix_inv(n, a)));
  __syncthreads();
  // backward: t_r -= L_jr t_j for r < j
  for (int j = n - 1; j >= 0; --j) {
    for (int r = w; r < j; r += EIG_WAVES) {
      FpRef T = num(M, ix_w(n, w, 0));
      fp_mul(c, T, num(M, ix_L(n, j, r)), num(M, ix_t(n, j)));
      fp_add(c, num(M, ix_t(n, r)), num(M, ix_t(n, r)), T, true);
    }
    __syncthreads();
  }
  for (int a = w; a < n; a += EIG_WAVES) fp_copy(c, num(M, ix_z(n, a)), num(M, ix_t(n, a)));
  __syncthreads();
}

// S_RQ = y'By / y'y
__device__ void eig_rayleigh(const EigMat& M, FpCtx c) {
  const int n = M.n, w = wave_id();
  // t_a = sum_b B_ab y_b
  for (int a = w; a < n; a += EIG_WAVES) {
    FpRef ta = num(M, ix_t(n, a));
    fp_set_zero(c, ta);
    wsync();
    FpRef T = num(M, ix_w(n, w, 0));
    for (int b = 0; b < n; ++b) {
      fp_mul(c, T, num(M, ix_B(n, a, b)), num(M, ix_y(n, b)));
      fp_add(c, ta, ta, T, false);
    }
  }
  __syncthreads();
  if (w == 0) {
    FpRef num_ = num(M, ix_s(n, S_NUM)), den = num(M, ix_s(n, S_DEN)), T = num(M, ix_w(n, 0, 0));
    fp_set_zero(c, num_);
    fp_set_zero(c, den);
    wsync();
    for (int a = 0; a < n; ++a) {
      fp_mul(c, T, num(M, ix_y(n, a)), num(M, ix_t(n, a)));
      fp_add(c, num_, num_, T, false);
      fp_mul(c, T, num(M, ix_y(n, a)), num(M, ix_y(n, a)));
      fp_add(c, den, den, T, false);
    }
    FpRef inv = num(M, ix_s(n, S_T1));
    fp_recip(c, inv, den, num(M, ix_w(n, 0, 1)), num(M, ix_w(n, 0, 2)));
    fp_mul(c, num(M, ix_s(n, S_RQ)), num_, inv);
  }
  __syncthreads();
}

// y = z * 2^-e, e = max exponent of z (exact)
__device__ void eig_normalise(const EigMat& M, FpCtx c, int* lds_int) {
  const int n = M.n, w = wave_id();
  if (threadIdx.x == 0) {
    int e = INT_MIN;
    for (int a = 0; a < n; ++a) {
      FpRef z = num(M, ix_z(n, a));
      if (!fp_is_zero(z) && z.hdr[1] > e) e = z.hdr[1];
    }
    lds_int[0] = e == INT_MIN ? 0 : e;
  }
  __syncthreads();
  const int e = lds_int[0];
  for (int a = w; a < n; a += EIG_WAVES) {
    FpRef y = num(M, ix_y(n, a));
    fp_copy(c, y, num(M, ix_z(n, a)));
    wsync();
    fp_ldexp(y, -e);
  }
  __syncthreads();
}

// number of bits the bracket resolves: exp(hi) - exp(hi - lo), capped
__device__ int eig_bits(const EigMat& M, FpCtx c) {
  const int n = M.n;
  FpRef W = num(M, ix_s(n, S_W));
  fp_add(c, W, num(M, ix_s(n, S_HI)), num(M, ix_s(n, S_LO)), true);
  if (fp_is_zero(W)) return 1 << 30;
  if (W.hdr[0] == 1) return -1;  // lo above hi: inconsistent
  return num(M, ix_s(n, S_HI)).hdr[1] - W.hdr[1];
}

__device__ void eig_body(const EigArgs& ea, int which) {
  const u32* __restrict__ blk = ea.blk;
  const int k = ea.k, nl = ea.nl, P = ea.P, NWM = ea.NWM;
  int* hdr_base = ea.hdr;
  u32* mant_base = ea.mant;
  const size_t nums_per = ea.nums_per;
  int* flags_base = ea.flags;
  DevStatus* st = ea.st;
  if (has_error(st)) return;
  // which = 0: k x k, 1: (k-1) x (k-1)
  const int n = k - which;
  if (n < 1) return;
  EigMat M;
  M.n = n;
  M.NWM = NWM;
  M.hdr = hdr_base + (size_t)which * nums_per * 2;
  M.mant = mant_base + (size_t)which * nums_per * NWM;
  M.flags = flags_base + which * 8;
  extern __shared__ u32 lds[];
  const int w = wave_id();
  int* lds_int = (int*)lds;
  FpCtx c;
  c.NWM = NWM;
  c.la = lds + 16 + w * 2 * (NWM + 8);
  c.lb = c.la + NWM + 8;
  const int NWF = NWM - 1;  // final working precision
  c.nw = NWF;
  // B from the integer block (full precision)
  for (int idx = w; idx < n * n; idx += EIG_WAVES) {
    const int a = idx / n, b = idx % n;
    fp_from_int(c, num(M, ix_B(n, a, b)), blk + ((size_t)a * k + b) * nl, nl);
  }
  __syncthreads();
  if (n == 1) {
    if (w == 0) fp_copy(c, num(M, ix_s(n, S_RES)), num(M, ix_B(n, 0, 0)));
    if (threadIdx.x == 0) M.flags[1] = 0;
    __syncthreads();
    goto finish;
  }
  {
    c.nw = 4 < NWF ? 4 : NWF;
    // hi = Gershgorin bound (1 + 2^-16), lo = max diagonal, y = 1
    if (w == 0) {
      FpRef hi = num(M, ix_s(n, S_HI)), lo = num(M, ix_s(n, S_LO));
      FpRef T = num(M, ix_w(n, 0, 0)), R = num(M, ix_w(n, 0, 1));
      FpCtx cf = c;
      cf.nw = NWF;
      fp_set_zero(cf, hi);
      fp_copy(cf, lo, num(M, ix_B(n, 0, 0)));
      wsync();
      for (int a = 0; a < n; ++a) {
        fp_set_zero(cf, R);
        wsync();
        for (int b = 0; b < n; ++b) {
          fp_copy(cf, T, num(M, ix_B(n, a, b)));
          wsync();
          if (lane_id() == 0 && T.hdr[0] == 1) T.hdr[0] = 0;  // |B_ab|
          wsync();
          fp_add(cf, R, R, T, false);
        }
        if (fp_cmp(cf, R, hi) > 0) fp_copy(cf, hi, R);
        wsync();
        if (fp_cmp(cf, num(M, ix_B(n, a, a)), lo) > 0) fp_copy(cf, lo, num(M, ix_B(n, a, a)));
        wsync();
      }
      // hi *= 1 + 2^-16
      fp_copy(cf, T, hi);
      wsync();
      fp_ldexp(T, -16);
      fp_add(cf, hi, hi, T, false);
    }
    for (int a = w; a < n; a += EIG_WAVES) {
      FpRef y = num(M, ix_y(n, a));
      for (int j = lane_id(); j < NWM; j += WAVE) y.m[j] = (j == NWM - 1) ? 0x80000000u : 0u;
      if (lane_id() == 0) {
        y.hdr[0] = 0;
        y.hdr[1] = 1;
      }
    }
    __syncthreads();
    const long target_bits = (long)P + 32;
    float cexp = 2.0f;  // log2 of the constant c in hi' = lo + c (hi - lo)^2 / hi
    int it = 0;
    bool have_factor = false;
    for (; it < ea.maxit; ++it) {
      if (!have_factor) {
        const bool pd = eig_factor(M, c, num(M, ix_s(n, S_HI)), lds_int + 4);
        if (!pd) {
          // hi was not above lambda_max at this precision: widen it
          if (w == 0) {
            FpRef hi = num(M, ix_s(n, S_HI)), lo = num(M, ix_s(n, S_LO)), T = num(M, ix_w(n, 0, 0));
            fp_add(c, T, hi, lo, true);  // hi - lo
            if (fp_is_zero(T) || T.hdr[0]) {
              fp_copy(c, T, hi);
              wsync();
              fp_ldexp(T, -20);
            }
            fp_add(c, hi, hi, T, false);
          }
          __syncthreads();
          continue;
        }
      }
      eig_solve(M, c);
      eig_normalise(M, c, lds_int + 8);
      eig_rayleigh(M, c);
      int bits;
      if (w == 0) {
        FpRef lo = num(M, ix_s(n, S_LO)), rq = num(M, ix_s(n, S_RQ));
        if (fp_cmp(c, rq, lo) > 0) fp_copy(c, lo, rq);
        wsync();
        bits = eig_bits(M, c);
        if (lane_id() == 0) lds_int[12] = bits;
      }
      __syncthreads();
      bits = lds_int[12];
      if (threadIdx.x == 0 && it < 24) flags_base[16 + which * 24 + it] = bits * 1000 + c.nw;
      if (bits < 0) {
        // the bounds crossed: at full precision that is rounding, the bracket
        // has closed; below it the iteration has gone wrong
        if (c.nw == NWF) break;
        if (threadIdx.x == 0) set_status(st, HL_ENOCONV, which);
        return;
      }
      if (bits >= target_bits && c.nw == NWF) break;
      // precision for the trial factorisation, which the next solve reuses: its
      // shift lies about 2^-2bits above lambda_max, so the system is that badly
      // conditioned and the solution must still carry 2 bits of accuracy
      long need = 4L * bits + 160;
      int nwn = (int)((need + 31) / 32);
      if (nwn < 4) nwn = 4;
      if (nwn > NWF) nwn = NWF;
      if (nwn > c.nw) c.nw = nwn;
      // trial upper bound: lo + c (hi - lo)^2 / hi, capped at lo + (hi - lo) / 2
      if (w == 0) {
        FpRef hi = num(M, ix_s(n, S_HI)), lo = num(M, ix_s(n, S_LO)), Wd = num(M, ix_s(n, S_W));
        FpRef T = num(M, ix_s(n, S_T1)), U = num(M, ix_s(n, S_T2)), tr = num(M, ix_s(n, S_TRY));
        fp_add(c, Wd, hi, lo, true);
        fp_mul(c, T, Wd, Wd);
        fp_recip(c, U, hi, num(M, ix_w(n, 0, 1)), num(M, ix_w(n, 0, 2)));
        fp_mul(c, T, T, U);
        const int ce = (int)cexp;
        fp_ldexp(T, ce);
        FpRef half = num(M, ix_s(n, S_T3));
        fp_copy(c, half, Wd);
        wsync();
        fp_ldexp(half, -1);
        if (fp_cmp(c, T, half) > 0) fp_copy(c, T, half);
        wsync();
        // not below what the working precision can add to lo
        fp_copy(c, half, hi);
        wsync();
        fp_ldexp(half, -(32 * c.nw - 40));
        if (fp_cmp(c, T, half) < 0) fp_copy(c, T, half);
        wsync();
        fp_add(c, tr, lo, T, false);
      }
      __syncthreads();
      const bool pd = eig_factor(M, c, num(M, ix_s(n, S_TRY)), lds_int + 4);
      if (w == 0) {
        if (pd) {
          fp_copy(c, num(M, ix_s(n, S_HI)), num(M, ix_s(n, S_TRY)));
        } else {
          fp_copy(c, num(M, ix_s(n, S_LO)), num(M, ix_s(n, S_TRY)));
        }
      }
      __syncthreads();
      if (pd) {
        have_factor = true;
        cexp = cexp - 4.0f > 2.0f ? cexp - 4.0f : 2.0f;
      } else {
        have_factor = false;
        cexp += 8.0f;
      }
    }
    if (threadIdx.x == 0) M.flags[1] = it;
    if (it >= ea.maxit) {
      if (threadIdx.x == 0) set_status(st, HL_ENOCONV, which);
      return;
    }
    if (w == 0) fp_copy(c, num(M, ix_s(n, S_RES)), num(M, ix_s(n, S_LO)));
    __syncthreads();
  }
finish:
  // lambda_1 (without the block exponent) = 1 / lambda_max
  if (w == 0) {
    c.nw = NWF;
    FpRef res = num(M, ix_s(n, S_RES));
    FpRef inv = num(M, ix_s(n, S_ONE));
    fp_recip(c, inv, res, num(M, ix_w(n, 0, 1)), num(M, ix_w(n, 0, 2)));
  }
}

__global__ __launch_bounds__(EIG_THREADS) void k_eig(EigArgs a) { eig_body(a, blockIdx.x); }

// batch: blockIdx.y is the instance
__global__ __launch_bounds__(EIG_THREADS) void k_eig_b(const EigArgs* __restrict__ tab) {
  eig_body(tab[blockIdx.y], blockIdx.x);
}

// difference of the two results: trunc = lam(k) - lam(k-1) (scaled equally)
__device__ void eig_diff_body(const EigArgs& ea) {
  const int k = ea.k, NWM = ea.NWM;
  int* hdr_base = ea.hdr;
  u32* mant_base = ea.mant;
  const size_t nums_per = ea.nums_per;
  DevStatus* st = ea.st;
  if (has_error(st) || k < 2) return;
  extern __shared__ u32 lds[];
  FpCtx c;
  c.NWM = NWM;
  c.nw = NWM - 1;
  c.la = lds;
  c.lb = lds + NWM + 8;
  EigMat A, B;
  A.n = k;
  A.NWM = NWM;
  A.hdr = hdr_base;
  A.mant = mant_base;
  B.n = k - 1;
  B.NWM = NWM;
  B.hdr = hdr_base + nums_per * 2;
  B.mant = mant_base + nums_per * NWM;
  FpRef r = num(A, ix_s(k, S_T3));
  fp_add(c, r, num(A, ix_s(k, S_ONE)), num(B, ix_s(k - 1, S_ONE)), true);
}

__global__ __launch_bounds__(64) void k_eig_diff(EigArgs a) { eig_diff_body(a); }
__global__ __launch_bounds__(64) void k_eig_diff_b(const EigArgs* __restrict__ tab) { eig_diff_body(tab[blockIdx.x]); }

// ---------------------------------------------------------------------------
// The same iteration, run from the host as a sequence of launches: every
// independent multiprecision product of a phase gets a workgroup of its own
// (EIG2_THREADS threads, the product formed by all its waves), so a step costs
// about one product's time instead of (products / waves) of them.  Each
// number sees exactly the operations, in the same order, as in k_eig, so the
// results are the same bits.  The host reads the bracket's state back at the
// two decision points of an iteration (positive definite?  bits resolved?).
constexpr int EIG2_THREADS = 256;

// workgroup context: wave scratch la, lb (NWM + 8 each), product (2 NWM),
// column sums (6 NWM)
struct WgCtx {
  FpCtx c;
  u32* pr;
  u32* cb;
};

__device__ __forceinline__ WgCtx wg_ctx(int NWM, int nw) {
  extern __shared__ u32 lds2[];
  WgCtx g;
  g.c.NWM = NWM;
  g.c.nw = nw;
  g.c.la = lds2 + 16;
  g.c.lb = g.c.la + NWM + 8;
  g.pr = g.c.lb + NWM + 8;
  g.cb = g.pr + 2 * NWM + 8;
  return g;
}

size_t eig2_lds_bytes(int NWM) { return (size_t)(16 + 2 * (NWM + 8) + 2 * NWM + 8 + 6 * NWM + 8) * 4; }

// z = x * y with every thread of the workgroup (the bits of fp_mul)
__device__ void wg_fp_mul(const WgCtx& g, FpRef z, const FpRef& x, const FpRef& y) {
  const FpCtx& c = g.c;
  const bool zero = fp_is_zero(x) || fp_is_zero(y);
  const int sx = x.hdr[0], sy = y.hdr[0], e = x.hdr[1] + y.hdr[1];
  __syncthreads();
  if (zero) {
    if (wave_id() == 0) fp_set_zero(c, z);
    __syncthreads();
    return;
  }
  const int nw = c.nw, top = c.NWM - nw;
  u32* A = c.la;
  u32* B = c.lb;
  for (int j = threadIdx.x; j < nw; j += blockDim.x) {
    A[j] = x.m[top + j];
    B[j] = y.m[top + j];
  }
  __syncthreads();
  // the exact product: int8 MFMA once the mantissas are long and its scratch
  // fits in the column-sum buffer (6 NWM words), else the vector-ALU scan
  if ((long)nw * nw >= 16384 && wm_scratch_bytes(nw, nw) <= (size_t)6 * c.NWM * 4)
    wg_mfma_mul(A, nw, B, nw, g.pr, 2 * nw, g.cb);
  else
    g_mul(A, nw, B, nw, g.pr, 2 * nw, g.cb);
  // product limbs nw-1 .. 2nw-1, normalised by at most one bit, to the top nw
  const u32* Q = g.pr + (nw - 1);
  const bool low = (Q[nw] >> 31) == 0;
  for (int j = threadIdx.x; j < c.NWM; j += blockDim.x) {
    u32 v = 0;
    if (j >= top) {
      const int i = j - top;  // 0 .. nw-1
      v = low ? ((Q[i + 1] << 1) | (Q[i] >> 31)) : Q[i + 1];
    }
    z.m[j] = v;
  }
  if (threadIdx.x == 0) {
    z.hdr[0] = sx ^ sy;
    z.hdr[1] = e - (low ? 1 : 0);
  }
  __threadfence_block();
  __syncthreads();
}

// wave 0 runs a wave operation, then the workgroup meets
#define WG_WAVE0(...)                   \
  do {                                  \
    if (wave_id() == 0) { __VA_ARGS__; } \
    __syncthreads();                    \
  } while (0)

// 1 / x as fp_recip does it, the products on the workgroup
__device__ void wg_fp_recip(const WgCtx& g0, FpRef z, const FpRef& x, FpRef t1, FpRef t2) {
  WgCtx g = g0;
  const FpCtx& c0 = g0.c;
  const u32 m1 = x.m[c0.NWM - 1], m0 = x.m[c0.NWM - 2];
  const u64 topv = ((u64)m1 << 32) | m0;
  const u64 top32 = topv >> 32;
  u64 q = (~0ull) / (top32 + 1);
  if (q < (1ull << 32)) q = 1ull << 32;
  const int xs = x.hdr[0], xe = x.hdr[1];
  __syncthreads();
  for (int j = threadIdx.x; j < c0.NWM; j += blockDim.x) {
    u32 v = 0;
    if (j == c0.NWM - 1) v = (u32)(q >> 1);
    if (j == c0.NWM - 2) v = (u32)(q << 31);
    z.m[j] = v;
  }
  if (threadIdx.x == 0) {
    z.hdr[0] = xs;
    z.hdr[1] = 1 - xe;
  }
  __threadfence_block();
  __syncthreads();
  const int target = c0.nw;
  int prec = 1;
  for (int it = 0; it < 40; ++it) {
    int np = 2 * prec;
    if (np > target) np = target;
    g.c.nw = np + 1 <= c0.NWM - 1 ? np + 1 : c0.NWM - 1;
    if (g.c.nw > target) g.c.nw = target;
    const int passes = (np >= target && it > 0 && np == target) ? 2 : 1;
    for (int pass = 0; pass < passes; ++pass) {
      wg_fp_mul(g, t1, x, z);
      WG_WAVE0({
        for (int j = lane_id(); j < g.c.NWM; j += WAVE) t2.m[j] = (j == g.c.NWM - 1) ? 0x80000000u : 0u;
        if (lane_id() == 0) {
          t2.hdr[0] = 0;
          t2.hdr[1] = 1;
        }
        wsync();
        fp_add(g.c, t2, t2, t1, true);
      });
      wg_fp_mul(g, t1, z, t2);
      WG_WAVE0(fp_add(g.c, z, z, t1, false));
    }
    prec = np;
    if (np >= target) break;
  }
}

__device__ __forceinline__ EigMat eig_mat(const EigArgs& ea, int which) {
  EigMat M;
  M.n = ea.k - (which & 1);
  M.NWM = ea.NWM;
  M.hdr = ea.hdr + (size_t)which * ea.nums_per * 2;
  M.mant = ea.mant + (size_t)which * ea.nums_per * ea.NWM;
  M.flags = ea.flags + eig_flag_off(which);
  return M;
}

// flags of a block: [0] status, [1] iterations, [2] positive definite, [3] bits
__global__ __launch_bounds__(64) void k_e2_init_b(EigArgs a, int which) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n;
  extern __shared__ u32 lds2[];
  FpCtx c;
  c.NWM = a.NWM;
  c.nw = a.NWM - 1;
  c.la = lds2;
  c.lb = lds2 + a.NWM + 8;
  const int idx = blockIdx.x;
  if (idx >= n * n) return;
  fp_from_int(c, num(M, ix_B(n, idx / n, idx % n)), a.blk + ((size_t)(idx / n) * a.k + (idx % n)) * a.nl, a.nl);
}

// hi = Gershgorin bound (1 + 2^-16), lo = max diagonal, y = 1 (as k_eig)
__global__ __launch_bounds__(64) void k_e2_init(EigArgs a, int which) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n;
  extern __shared__ u32 lds2[];
  FpCtx cf;
  cf.NWM = a.NWM;
  cf.nw = a.NWM - 1;
  cf.la = lds2;
  cf.lb = lds2 + a.NWM + 8;
  if (n == 1) {
    fp_copy(cf, num(M, ix_s(n, S_RES)), num(M, ix_B(n, 0, 0)));
    if (lane_id() == 0) M.flags[1] = 0;
    return;
  }
  FpRef hi = num(M, ix_s(n, S_HI)), lo = num(M, ix_s(n, S_LO));
  FpRef T = num(M, ix_w(n, 0, 0)), R = num(M, ix_w(n, 0, 1));
  fp_set_zero(cf, hi);
  fp_copy(cf, lo, num(M, ix_B(n, 0, 0)));
  wsync();
  for (int ia = 0; ia < n; ++ia) {
    fp_set_zero(cf, R);
    wsync();
    for (int ib = 0; ib < n; ++ib) {
      fp_copy(cf, T, num(M, ix_B(n, ia, ib)));
      wsync();
      if (lane_id() == 0 && T.hdr[0] == 1) T.hdr[0] = 0;
      wsync();
      fp_add(cf, R, R, T, false);
    }
    if (fp_cmp(cf, R, hi) > 0) fp_copy(cf, hi, R);
    wsync();
    if (fp_cmp(cf, num(M, ix_B(n, ia, ia)), lo) > 0) fp_copy(cf, lo, num(M, ix_B(n, ia, ia)));
    wsync();
  }
  fp_copy(cf, T, hi);
  wsync();
  fp_ldexp(T, -16);
  fp_add(cf, hi, hi, T, false);
  for (int ia = 0; ia < n; ++ia) {
    FpRef y = num(M, ix_y(n, ia));
    for (int j = lane_id(); j < a.NWM; j += WAVE) y.m[j] = (j == a.NWM - 1) ? 0x80000000u : 0u;
    if (lane_id() == 0) {
      y.hdr[0] = 0;
      y.hdr[1] = 1;
    }
  }
  wsync();
}

// C = sigma I - B (one wave per entry)
__global__ __launch_bounds__(64) void k_e2_shift(EigArgs a, int which, int nw, int sig) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n, idx = blockIdx.x;
  extern __shared__ u32 lds2[];
  FpCtx c;
  c.NWM = a.NWM;
  c.nw = nw;
  c.la = lds2;
  c.lb = lds2 + a.NWM + 8;
  const int ia = idx / n, ib = idx % n;
  FpRef C = num(M, ix_C(n, ia, ib));
  FpRef B = num(M, ix_B(n, ia, ib));
  if (ia == ib) {
    fp_add(c, C, num(M, ix_s(n, sig)), B, true);
  } else {
    fp_copy(c, C, B);
    wsync();
    if (lane_id() == 0 && C.hdr[0] != FPZERO_TAG) C.hdr[0] ^= 1;
  }
  if (idx == 0 && lane_id() == 0) M.flags[2] = 1;
}

// pivot i: positive?  inv_i = 1 / C_ii
__global__ __launch_bounds__(EIG2_THREADS) void k_e2_pivot(EigArgs a, int which, int nw, int i) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n;
  if (!M.flags[2]) return;
  const WgCtx g = wg_ctx(a.NWM, nw);
  FpRef d = num(M, ix_C(n, i, i));
  const bool pos = !fp_is_zero(d) && d.hdr[0] == 0;
  __syncthreads();
  if (!pos) {
    if (threadIdx.x == 0) M.flags[2] = 0;
    return;
  }
  wg_fp_recip(g, num(M, ix_inv(n, i)), d, num(M, ix_w(n, 0, 0)), num(M, ix_w(n, 0, 1)));
}

// L_ri = C_ri inv_i, r = i + 1 + blockIdx.x
__global__ __launch_bounds__(EIG2_THREADS) void k_e2_lcol(EigArgs a, int which, int nw, int i) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n, r = i + 1 + blockIdx.x;
  if (!M.flags[2] || r >= n) return;
  const WgCtx g = wg_ctx(a.NWM, nw);
  wg_fp_mul(g, num(M, ix_L(n, r, i)), num(M, ix_C(n, r, i)), num(M, ix_inv(n, i)));
}

// C_rc -= L_ri C_ci for r >= c > i (one workgroup per pair)
__global__ __launch_bounds__(EIG2_THREADS) void k_e2_update(EigArgs a, int which, int nw, int i) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n;
  if (!M.flags[2]) return;
  // pair index p -> (r, c) with i < c <= r < n, row by row
  const int p = blockIdx.x;
  int rr = 0;
  while ((rr + 1) * (rr + 2) / 2 <= p) ++rr;
  const int r = i + 1 + rr, cc = i + 1 + (p - rr * (rr + 1) / 2);
  if (r >= n) return;
  const WgCtx g = wg_ctx(a.NWM, nw);
  FpRef T = num(M, ix_T(n, r, cc));
  wg_fp_mul(g, T, num(M, ix_L(n, r, i)), num(M, ix_C(n, cc, i)));
  WG_WAVE0(fp_add(g.c, num(M, ix_C(n, r, cc)), num(M, ix_C(n, r, cc)), T, true));
}

// vector copies: mode 0 t = y, 1 z = t
__global__ __launch_bounds__(64) void k_e2_copy(EigArgs a, int which, int nw, int mode) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n, ia = blockIdx.x;
  if (ia >= n) return;
  FpCtx c;
  c.NWM = a.NWM;
  c.nw = nw;
  if (mode == 0) fp_copy(c, num(M, ix_t(n, ia)), num(M, ix_y(n, ia)));
  else fp_copy(c, num(M, ix_z(n, ia)), num(M, ix_t(n, ia)));
}

// forward (dir 0): t_r -= L_rj t_j, r > j;  backward (dir 1): t_r -= L_jr t_j, r < j
__global__ __launch_bounds__(EIG2_THREADS) void k_e2_sweep(EigArgs a, int which, int nw, int j, int dir) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n;
  const int r = dir == 0 ? j + 1 + blockIdx.x : blockIdx.x;
  if (dir == 0 ? r >= n : r >= j) return;
  const WgCtx g = wg_ctx(a.NWM, nw);
  FpRef T = num(M, ix_T(n, r, 0));
  if (dir == 0) wg_fp_mul(g, T, num(M, ix_L(n, r, j)), num(M, ix_t(n, j)));
  else wg_fp_mul(g, T, num(M, ix_L(n, j, r)), num(M, ix_t(n, j)));
  WG_WAVE0(fp_add(g.c, num(M, ix_t(n, r)), num(M, ix_t(n, r)), T, true));
}

// t_a *= inv_a
__global__ __launch_bounds__(EIG2_THREADS) void k_e2_scale(EigArgs a, int which, int nw) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n, ia = blockIdx.x;
  if (ia >= n) return;
  const WgCtx g = wg_ctx(a.NWM, nw);
  wg_fp_mul(g, num(M, ix_t(n, ia)), num(M, ix_t(n, ia)), num(M, ix_inv(n, ia)));
}

// y = z 2^-e (as eig_normalise)
__global__ __launch_bounds__(64) void k_e2_normalise(EigArgs a, int which, int nw) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n;
  FpCtx c;
  c.NWM = a.NWM;
  c.nw = nw;
  int e = INT_MIN;
  for (int ia = 0; ia < n; ++ia) {
    FpRef z = num(M, ix_z(n, ia));
    if (!fp_is_zero(z) && z.hdr[1] > e) e = z.hdr[1];
  }
  if (e == INT_MIN) e = 0;
  for (int ia = 0; ia < n; ++ia) {
    FpRef y = num(M, ix_y(n, ia));
    fp_copy(c, y, num(M, ix_z(n, ia)));
    wsync();
    fp_ldexp(y, -e);
  }
}

// Rayleigh quotient, products: P_ab = B_ab y_b (mode 0), then U_a = y_a t_a,
// V_a = y_a y_a (mode 1, blockIdx.x = 2a + {0, 1})
__global__ __launch_bounds__(EIG2_THREADS) void k_e2_rq_prod(EigArgs a, int which, int nw, int mode) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n, idx = blockIdx.x;
  const WgCtx g = wg_ctx(a.NWM, nw);
  if (mode == 0) {
    if (idx >= n * n) return;
    const int ia = idx / n, ib = idx % n;
    wg_fp_mul(g, num(M, ix_T(n, ia, ib)), num(M, ix_B(n, ia, ib)), num(M, ix_y(n, ib)));
  } else {
    if (idx >= 2 * n) return;
    const int ia = idx >> 1;
    if (idx & 1) wg_fp_mul(g, num(M, ix_T(n, ia, 1)), num(M, ix_y(n, ia)), num(M, ix_y(n, ia)));
    else wg_fp_mul(g, num(M, ix_T(n, ia, 0)), num(M, ix_y(n, ia)), num(M, ix_t(n, ia)));
  }
}

// t_a = sum_b P_ab in order b = 0 .. n-1
__global__ __launch_bounds__(64) void k_e2_rq_rows(EigArgs a, int which, int nw) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n, ia = blockIdx.x;
  if (ia >= n) return;
  extern __shared__ u32 lds2[];
  FpCtx c;
  c.NWM = a.NWM;
  c.nw = nw;
  c.la = lds2;
  c.lb = lds2 + a.NWM + 8;
  FpRef ta = num(M, ix_t(n, ia));
  fp_set_zero(c, ta);
  wsync();
  for (int ib = 0; ib < n; ++ib) fp_add(c, ta, ta, num(M, ix_T(n, ia, ib)), false);
}

// num = sum U_a, den = sum V_a (in the order of eig_rayleigh), RQ = num / den,
// lo = max(lo, RQ), bits, trace
__global__ __launch_bounds__(EIG2_THREADS) void k_e2_rq_final(EigArgs a, int which, int nw, int it) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n;
  const WgCtx g = wg_ctx(a.NWM, nw);
  FpRef num_ = num(M, ix_s(n, S_NUM)), den = num(M, ix_s(n, S_DEN));
  WG_WAVE0({
    fp_set_zero(g.c, num_);
    fp_set_zero(g.c, den);
    wsync();
    for (int ia = 0; ia < n; ++ia) {
      fp_add(g.c, num_, num_, num(M, ix_T(n, ia, 0)), false);
      fp_add(g.c, den, den, num(M, ix_T(n, ia, 1)), false);
    }
  });
  FpRef inv = num(M, ix_s(n, S_T1));
  wg_fp_recip(g, inv, den, num(M, ix_w(n, 0, 1)), num(M, ix_w(n, 0, 2)));
  wg_fp_mul(g, num(M, ix_s(n, S_RQ)), num_, inv);
  WG_WAVE0({
    FpRef lo = num(M, ix_s(n, S_LO)), rq = num(M, ix_s(n, S_RQ));
    if (fp_cmp(g.c, rq, lo) > 0) fp_copy(g.c, lo, rq);
    wsync();
    const int bits = eig_bits(M, g.c);
    if (lane_id() == 0) {
      M.flags[3] = bits;
      if (it < 24 && which < 2) a.flags[16 + which * 24 + it] = bits * 1000 + nw;
    }
  });
}

// trial upper bound lo + c (hi - lo)^2 / hi, capped at lo + (hi - lo) / 2 and
// floored at hi 2^-(32 nw - 40) (as k_eig)
__global__ __launch_bounds__(EIG2_THREADS) void k_e2_trial(EigArgs a, int which, int nw, int cexp) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n;
  const WgCtx g = wg_ctx(a.NWM, nw);
  FpRef hi = num(M, ix_s(n, S_HI)), lo = num(M, ix_s(n, S_LO)), Wd = num(M, ix_s(n, S_W));
  FpRef T = num(M, ix_s(n, S_T1)), U = num(M, ix_s(n, S_T2)), tr = num(M, ix_s(n, S_TRY));
  WG_WAVE0(fp_add(g.c, Wd, hi, lo, true));
  wg_fp_mul(g, T, Wd, Wd);
  wg_fp_recip(g, U, hi, num(M, ix_w(n, 0, 1)), num(M, ix_w(n, 0, 2)));
  wg_fp_mul(g, T, T, U);
  WG_WAVE0({
    fp_ldexp(T, cexp);
    FpRef half = num(M, ix_s(n, S_T3));
    fp_copy(g.c, half, Wd);
    wsync();
    fp_ldexp(half, -1);
    if (fp_cmp(g.c, T, half) > 0) fp_copy(g.c, T, half);
    wsync();
    fp_copy(g.c, half, hi);
    wsync();
    fp_ldexp(half, -(32 * nw - 40));
    if (fp_cmp(g.c, T, half) < 0) fp_copy(g.c, T, half);
    wsync();
    fp_add(g.c, tr, lo, T, false);
  });
}

// mode 0: after the trial factorisation, hi = trial (positive definite) or
// lo = trial; mode 1: widen hi (the factorisation at hi failed); mode 2: the
// result lo; mode 3: iterations
__global__ __launch_bounds__(64) void k_e2_control(EigArgs a, int which, int nw, int mode, int val) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n;
  extern __shared__ u32 lds2[];
  FpCtx c;
  c.NWM = a.NWM;
  c.nw = nw;
  c.la = lds2;
  c.lb = lds2 + a.NWM + 8;
  if (mode == 0) {
    if (M.flags[2]) fp_copy(c, num(M, ix_s(n, S_HI)), num(M, ix_s(n, S_TRY)));
    else fp_copy(c, num(M, ix_s(n, S_LO)), num(M, ix_s(n, S_TRY)));
  } else if (mode == 1) {
    FpRef hi = num(M, ix_s(n, S_HI)), lo = num(M, ix_s(n, S_LO)), T = num(M, ix_w(n, 0, 0));
    fp_add(c, T, hi, lo, true);
    if (fp_is_zero(T) || T.hdr[0]) {
      fp_copy(c, T, hi);
      wsync();
      fp_ldexp(T, -20);
    }
    fp_add(c, hi, hi, T, false);
  } else if (mode == 2) {
    fp_copy(c, num(M, ix_s(n, S_RES)), num(M, ix_s(n, S_LO)));
  } else if (lane_id() == 0) {
    M.flags[1] = val;
  }
}

// lambda_1 (without the block exponent) = 1 / lambda_max
__global__ __launch_bounds__(EIG2_THREADS) void k_e2_finish(EigArgs a, int which) {
  const EigMat M = eig_mat(a, which);
  const int n = M.n;
  const WgCtx g = wg_ctx(a.NWM, a.NWM - 1);
  wg_fp_recip(g, num(M, ix_s(n, S_ONE)), num(M, ix_s(n, S_RES)), num(M, ix_w(n, 0, 1)), num(M, ix_w(n, 0, 2)));
}

// ---------------------------------------------------------------------------
// The next eigenvalues (lambda_2, lambda_3 of Table 2) by deflation: matrix
// `which` (2 or more) is matrix which - 2 less its converged eigenpair,
// B' = B - mu y y^T / (y^T y).  For symmetric B this keeps every other eigenpair
// and sends mu to 0, so the largest eigenvalue of B' is the next one of B; an
// error e in the eigenvector y moves it by O(mu e^2) only.  Step 1 (one
// workgroup): g_a = (mu / y^T y) y_a, into the destination's vector t.
__global__ __launch_bounds__(EIG2_THREADS) void k_e2_defl_vec(EigArgs a, int which) {
  const EigMat S = eig_mat(a, which - 2), D = eig_mat(a, which);
  const int n = D.n;
  const WgCtx g = wg_ctx(a.NWM, a.NWM - 1);
  for (int ia = 0; ia < n; ++ia) wg_fp_mul(g, num(D, ix_T(n, ia, 0)), num(S, ix_y(n, ia)), num(S, ix_y(n, ia)));
  FpRef den = num(D, ix_s(n, S_DEN)), inv = num(D, ix_s(n, S_T1)), f = num(D, ix_s(n, S_T2));
  WG_WAVE0({
    fp_set_zero(g.c, den);
    wsync();
    for (int ia = 0; ia < n; ++ia) fp_add(g.c, den, den, num(D, ix_T(n, ia, 0)), false);
  });
  wg_fp_recip(g, inv, den, num(D, ix_w(n, 0, 1)), num(D, ix_w(n, 0, 2)));
  wg_fp_mul(g, f, num(S, ix_s(n, S_RES)), inv);
  for (int ia = 0; ia < n; ++ia) wg_fp_mul(g, num(D, ix_t(n, ia)), f, num(S, ix_y(n, ia)));
}

// Step 2 (one workgroup per pair a >= b): B'_ab = B_ab - g_a y_b, copied to
// B'_ba so that B' stays exactly symmetric
__global__ __launch_bounds__(EIG2_THREADS) void k_e2_defl_mat(EigArgs a, int which) {
  const EigMat S = eig_mat(a, which - 2), D = eig_mat(a, which);
  const int n = D.n, p = blockIdx.x;
  int ia = 0;
  while ((ia + 1) * (ia + 2) / 2 <= p) ++ia;
  const int ib = p - ia * (ia + 1) / 2;
  if (ia >= n) return;
  const WgCtx g = wg_ctx(a.NWM, a.NWM - 1);
  FpRef T = num(D, ix_T(n, ia, ib));
  wg_fp_mul(g, T, num(D, ix_t(n, ia)), num(S, ix_y(n, ib)));
  WG_WAVE0({
    fp_add(g.c, num(D, ix_B(n, ia, ib)), num(S, ix_B(n, ia, ib)), T, true);
    wsync();
    if (ia != ib) fp_copy(g.c, num(D, ix_B(n, ib, ia)), num(D, ix_B(n, ia, ib)));
  });
}

// trunc_j = 1 / mu_j(k) - 1 / mu_j(k - 1) into the scalar T3 of matrix `which` (even)
__global__ __launch_bounds__(64) void k_e2_diff(EigArgs a, int which) {
  const EigMat A = eig_mat(a, which), B = eig_mat(a, which + 1);
  extern __shared__ u32 lds2[];
  FpCtx c;
  c.NWM = a.NWM;
  c.nw = a.NWM - 1;
  c.la = lds2;
  c.lb = lds2 + a.NWM + 8;
  fp_add(c, num(A, ix_s(A.n, S_T3)), num(A, ix_s(A.n, S_ONE)), num(B, ix_s(B.n, S_ONE)), true);
}

namespace {
int read_flag(const EigArgs& a, int which, int slot, hipStream_t st, hipError_t* err) {
  int v = 0;
  *err = hipMemcpyAsync(&v, a.flags + eig_flag_off(which) + slot, 4, hipMemcpyDeviceToHost, st);
  if (*err == hipSuccess) *err = hipStreamSynchronize(st);
  return v;
}
}  // namespace

#define E2CHK(x)                           \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) return e_;       \
  } while (0)

// one block (which = 0: k x k, 1: (k-1) x (k-1)); *conv = 0 if it did not converge
static hipError_t eig2_block(const EigArgs& a, int which, hipStream_t st, int* conv) {
  const int n = a.k - (which & 1), NWM = a.NWM, NWF = NWM - 1;
  const size_t lw = (size_t)2 * (NWM + 8) * 4;   // one wave's scratch
  const size_t lg = eig2_lds_bytes(NWM);
  *conv = 1;
  if (which < 2) {  // deflated matrices are written by k_e2_defl_mat
    hipLaunchKernelGGL(k_e2_init_b, dim3(n * n), dim3(64), lw, st, a, which);
    E2CHK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_e2_init, dim3(1), dim3(64), lw, st, a, which);
  E2CHK(hipGetLastError());
  if (n > 1) {
    const long target_bits = (long)a.P + 32;
    int nw = 4 < NWF ? 4 : NWF;
    float cexp = 2.0f;
    bool have_factor = false;
    hipError_t err = hipSuccess;
    auto factor = [&](int sig) -> hipError_t {
      hipLaunchKernelGGL(k_e2_shift, dim3(n * n), dim3(64), lw, st, a, which, nw, sig);
      E2CHK(hipGetLastError());
      for (int i = 0; i < n; ++i) {
        hipLaunchKernelGGL(k_e2_pivot, dim3(1), dim3(EIG2_THREADS), lg, st, a, which, nw, i);
        E2CHK(hipGetLastError());
        const int m = n - i - 1;
        if (m > 0) {
          hipLaunchKernelGGL(k_e2_lcol, dim3(m), dim3(EIG2_THREADS), lg, st, a, which, nw, i);
          E2CHK(hipGetLastError());
          hipLaunchKernelGGL(k_e2_update, dim3(m * (m + 1) / 2), dim3(EIG2_THREADS), lg, st, a, which, nw, i);
          E2CHK(hipGetLastError());
        }
      }
      return hipSuccess;
    };
    int it = 0;
    for (; it < a.maxit; ++it) {
      if (!have_factor) {
        E2CHK(factor(S_HI));
        const int pd = read_flag(a, which, 2, st, &err);
        E2CHK(err);
        if (!pd) {
          hipLaunchKernelGGL(k_e2_control, dim3(1), dim3(64), lw, st, a, which, nw, 1, 0);
          E2CHK(hipGetLastError());
          continue;
        }
      }
      // z = C^-1 y, y = normalised z, Rayleigh quotient
      hipLaunchKernelGGL(k_e2_copy, dim3(n), dim3(64), 0, st, a, which, nw, 0);
      for (int j = 0; j < n - 1; ++j)
        hipLaunchKernelGGL(k_e2_sweep, dim3(n - j - 1), dim3(EIG2_THREADS), lg, st, a, which, nw, j, 0);
      hipLaunchKernelGGL(k_e2_scale, dim3(n), dim3(EIG2_THREADS), lg, st, a, which, nw);
      for (int j = n - 1; j >= 1; --j)
        hipLaunchKernelGGL(k_e2_sweep, dim3(j), dim3(EIG2_THREADS), lg, st, a, which, nw, j, 1);
      hipLaunchKernelGGL(k_e2_copy, dim3(n), dim3(64), 0, st, a, which, nw, 1);
      hipLaunchKernelGGL(k_e2_normalise, dim3(1), dim3(64), 0, st, a, which, nw);
      hipLaunchKernelGGL(k_e2_rq_prod, dim3(n * n), dim3(EIG2_THREADS), lg, st, a, which, nw, 0);
      hipLaunchKernelGGL(k_e2_rq_rows, dim3(n), dim3(64), lw, st, a, which, nw);
      hipLaunchKernelGGL(k_e2_rq_prod, dim3(2 * n), dim3(EIG2_THREADS), lg, st, a, which, nw, 1);
      hipLaunchKernelGGL(k_e2_rq_final, dim3(1), dim3(EIG2_THREADS), lg, st, a, which, nw, it);
      E2CHK(hipGetLastError());
      const int bits = read_flag(a, which, 3, st, &err);
      E2CHK(err);
      if (bits < 0) {
        if (nw == NWF) break;
        *conv = 0;
        return hipSuccess;
      }
      if (bits >= target_bits && nw == NWF) break;
      long need = 4L * bits + 160;
      int nwn = (int)((need + 31) / 32);
      if (nwn < 4) nwn = 4;
      if (nwn > NWF) nwn = NWF;
      if (nwn > nw) nw = nwn;
      hipLaunchKernelGGL(k_e2_trial, dim3(1), dim3(EIG2_THREADS), lg, st, a, which, nw, (int)cexp);
      E2CHK(hipGetLastError());
      E2CHK(factor(S_TRY));
      hipLaunchKernelGGL(k_e2_control, dim3(1), dim3(64), lw, st, a, which, nw, 0, 0);
      E2CHK(hipGetLastError());
      const int pd = read_flag(a, which, 2, st, &err);
      E2CHK(err);
      if (pd) {
        have_factor = true;
        cexp = cexp - 4.0f > 2.0f ? cexp - 4.0f : 2.0f;
      } else {
        have_factor = false;
        cexp += 8.0f;
      }
    }
    hipLaunchKernelGGL(k_e2_control, dim3(1), dim3(64), lw, st, a, which, nw, 3, it);
    E2CHK(hipGetLastError());
    if (it >= a.maxit) {
      *conv = 0;
      return hipSuccess;
    }
    hipLaunchKernelGGL(k_e2_control, dim3(1), dim3(64), lw, st, a, which, nw, 2, 0);
    E2CHK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_e2_finish, dim3(1), dim3(EIG2_THREADS), lg, st, a, which);
  return hipGetLastError();
}

// dynamic LDS above the default for the workgroup kernels
static hipError_t eig2_attrs(size_t lg) {
  const void* big[] = {(const void*)k_e2_pivot,   (const void*)k_e2_lcol,     (const void*)k_e2_update,
                       (const void*)k_e2_sweep,   (const void*)k_e2_scale,    (const void*)k_e2_rq_prod,
                       (const void*)k_e2_rq_final, (const void*)k_e2_trial,   (const void*)k_e2_finish,
                       (const void*)k_e2_defl_vec, (const void*)k_e2_defl_mat};
  if (lg > 65536)
    for (const void* f : big) E2CHK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lg));
  return hipSuccess;
}

// *stop = the status word holds a device error from an earlier stage
static hipError_t eig2_status(DevStatus* st, hipStream_t stream, bool* stop) {
  unsigned long long sw = 0;
  E2CHK(hipMemcpyAsync(&sw, st, 8, hipMemcpyDeviceToHost, stream));
  E2CHK(hipStreamSynchronize(stream));
  *stop = sw != 0;
  return hipSuccess;
}

static hipError_t eig2_noconv(DevStatus* st, int which, hipStream_t stream) {
  const unsigned long long v = ((unsigned long long)HL_ENOCONV << 32) | (unsigned)which;
  E2CHK(hipMemcpyAsync(st, &v, 8, hipMemcpyHostToDevice, stream));
  return hipStreamSynchronize(stream);
}

// Host-driven eigen-step of both blocks; ENOCONV goes to the status word.  With
// a second stream the (k-1) x (k-1) block runs on it from a second host thread
// while the k x k block runs on the caller's: their launches are small and
// their workspace regions disjoint, so the two iterations overlap.
hipError_t launch_eig_host(const u32* blk, const Dims& dm, void* eig_ws, DevStatus* st, hipStream_t stream,
                           hipStream_t aux, int maxit) {
  EigArgs a = eig_args(blk, dm, eig_ws, st);
  if (maxit > 0) a.maxit = maxit;
  E2CHK(eig2_attrs(eig2_lds_bytes(a.NWM)));
  bool stop = false;
  E2CHK(eig2_status(st, stream, &stop));
  if (stop) return hipSuccess;
  const int nb = dm.k >= 2 ? 2 : 1;
  int conv[2] = {1, 1};
  if (nb == 2 && aux) {
    int dev = 0;
    E2CHK(hipGetDevice(&dev));
    hipEvent_t ev = nullptr;
    E2CHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e1 = hipEventRecord(ev, stream);   // the block is ready on the caller's stream
    if (e1 == hipSuccess) e1 = hipStreamWaitEvent(aux, ev, 0);
    if (e1 != hipSuccess) {
      (void)hipEventDestroy(ev);
      return e1;
    }
    std::thread other([&]() {
      e1 = hipSetDevice(dev);
      if (e1 == hipSuccess) e1 = eig2_block(a, 1, aux, &conv[1]);
      if (e1 == hipSuccess) e1 = hipEventRecord(ev, aux);
    });
    const hipError_t e0 = eig2_block(a, 0, stream, &conv[0]);
    other.join();
    if (e1 == hipSuccess) e1 = hipStreamWaitEvent(stream, ev, 0);
    (void)hipEventDestroy(ev);
    E2CHK(e0);
    E2CHK(e1);
  } else {
    for (int which = 0; which < nb; ++which) {
      E2CHK(eig2_block(a, which, stream, &conv[which]));
      if (!conv[which]) break;
    }
  }
  for (int which = 0; which < nb; ++which)
    if (!conv[which]) return eig2_noconv(st, which, stream);
  hipLaunchKernelGGL(k_eig_diff, dim3(1), dim3(64), (size_t)2 * (a.NWM + 8) * 4, stream, a);
  return hipGetLastError();
}

// The next `count` eigenvalues of both blocks by deflation (matrices 2 .. 2 count
// + 1), after launch_eig_host on the same workspace; needs k >= count + 2 and
// count <= EIG_MATS / 2 - 1 (checked by the caller).
hipError_t launch_eig_next(const u32* blk, const Dims& dm, void* eig_ws, int count, DevStatus* st,
                           hipStream_t stream) {
  const EigArgs a = eig_args(blk, dm, eig_ws, st);
  const size_t lg = eig2_lds_bytes(a.NWM);
  E2CHK(eig2_attrs(lg));
  bool stop = false;
  E2CHK(eig2_status(st, stream, &stop));
  if (stop) return hipSuccess;
  for (int j = 1; j <= count; ++j) {
    for (int h = 0; h < 2; ++h) {
      const int which = 2 * j + h, n = dm.k - h;
      hipLaunchKernelGGL(k_e2_defl_vec, dim3(1), dim3(EIG2_THREADS), lg, stream, a, which);
      E2CHK(hipGetLastError());
      hipLaunchKernelGGL(k_e2_defl_mat, dim3(n * (n + 1) / 2), dim3(EIG2_THREADS), lg, stream, a, which);
      E2CHK(hipGetLastError());
      int conv = 1;
      E2CHK(eig2_block(a, which, stream, &conv));
      if (!conv) return eig2_noconv(st, which, stream);
    }
    hipLaunchKernelGGL(k_e2_diff, dim3(1), dim3(64), (size_t)2 * (a.NWM + 8) * 4, stream, a, 2 * j);
    E2CHK(hipGetLastError());
  }
  return hipSuccess;
}

size_t eig_ws_bytes(const Dims& dm) {
  const int NWM = dm.nl + 4;
  const size_t per = (size_t)eig_numbers(dm.k);
  return EIG_MATS * per * (2 * 4 + (size_t)NWM * 4) + EIG_FLAG_INTS * 4;
}

// host: run the eigen-step on both blocks and read back the results
EigArgs eig_args(const u32* blk, const Dims& dm, void* eig_ws, DevStatus* st) {
  EigArgs a{};
  a.blk = blk;
  a.k = dm.k;
  a.nl = dm.nl;
  a.P = dm.P;
  a.NWM = dm.nl + 4;
  a.nums_per = (size_t)eig_numbers(dm.k);
  a.flags = (int*)eig_ws;
  a.hdr = a.flags + EIG_FLAG_INTS;
  a.mant = (u32*)(a.hdr + 2 * EIG_MATS * a.nums_per);
  a.st = st;
  a.maxit = EIG_MAXIT;
  return a;
}

static size_t eig_lds(int NWM) { return (size_t)(16 + EIG_WAVES * 2 * (NWM + 8)) * 4; }

hipError_t launch_eig(const u32* blk, const Dims& dm, void* eig_ws, DevStatus* st, hipStream_t stream) {
  const EigArgs a = eig_args(blk, dm, eig_ws, st);
  const size_t lds = eig_lds(a.NWM);
  if (lds > 65536) {
    hipError_t e0 = hipFuncSetAttribute((const void*)k_eig, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e0 != hipSuccess) return e0;
  }
  hipLaunchKernelGGL(k_eig, dim3(dm.k >= 2 ? 2 : 1), dim3(EIG_THREADS), lds, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_eig_diff, dim3(1), dim3(64), (size_t)2 * (a.NWM + 8) * 4, stream, a);
  return hipGetLastError();
}

hipError_t launch_eig_batch(const EigArgs* tab, int count, int nl_max, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const size_t lds = eig_lds(nl_max + 4);
  if (lds > 65536) {
    hipError_t e0 = hipFuncSetAttribute((const void*)k_eig_b, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e0 != hipSuccess) return e0;
  }
  hipLaunchKernelGGL(k_eig_b, dim3(2, count), dim3(EIG_THREADS), lds, stream, tab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_eig_diff_b, dim3(count), dim3(64), (size_t)2 * (nl_max + 4 + 8) * 4, stream, tab);
  return hipGetLastError();
}

// location of the k x k block's eigenvector (k numbers, consecutive headers and
// mantissas), left by the last iteration
void eig_vector_refs(const Dims& dm, void* eig_ws, int** hdr_out, u32** mant_out) {
  const int NWM = dm.nl + 4;
  const size_t per = (size_t)eig_numbers(dm.k);
  int* flags = (int*)eig_ws;
  int* hdr = flags + EIG_FLAG_INTS;
  u32* mant = (u32*)(hdr + 2 * EIG_MATS * per);
  *hdr_out = hdr + 2 * ix_y(dm.k, 0);
  *mant_out = mant + (size_t)ix_y(dm.k, 0) * NWM;
}

// locations of the results (host side arithmetic on offsets only)
void eig_result_refs(const Dims& dm, void* eig_ws, int which, int** hdr_out, u32** mant_out) {
  const int NWM = dm.nl + 4;
  const size_t per = (size_t)eig_numbers(dm.k);
  int* flags = (int*)eig_ws;
  int* hdr = flags + EIG_FLAG_INTS;
  u32* mant = (u32*)(hdr + 2 * EIG_MATS * per);
  // which: 0 -> 1/lambda_max(k), 1 -> 1/lambda_max(k-1), 2 -> difference, 3 -> iteration flags
  const int n = which == 1 ? dm.k - 1 : dm.k;
  const int blkidx = which == 1 ? 1 : 0;
  const int idx = which == 2 ? ix_s(n, S_T3) : ix_s(n, S_ONE);
  *hdr_out = hdr + (size_t)blkidx * per * 2 + 2 * idx;
  *mant_out = mant + ((size_t)blkidx * per + idx) * NWM;
}

// results of the deflated matrices: 1 / mu of matrix `mat`, or (diff, even
// mat) the difference left by k_e2_diff
void eig_next_refs(const Dims& dm, void* eig_ws, int mat, bool diff, int** hdr_out, u32** mant_out) {
  const int NWM = dm.nl + 4;
  const size_t per = (size_t)eig_numbers(dm.k);
  int* flags = (int*)eig_ws;
  int* hdr = flags + EIG_FLAG_INTS;
  u32* mant = (u32*)(hdr + 2 * EIG_MATS * per);
  const int n = dm.k - (mat & 1);
  const int idx = diff ? ix_s(n, S_T3) : ix_s(n, S_ONE);
  *hdr_out = hdr + (size_t)mat * per * 2 + 2 * idx;
  *mant_out = mant + ((size_t)mat * per + idx) * NWM;
}

// iterations used on matrix `mat`
int* eig_iter_ref(void* eig_ws, int mat) { return (int*)eig_ws + eig_flag_off(mat) + 1; }

}  // namespace hl
