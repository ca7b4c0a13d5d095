// First k columns of L^-1 (Algorithm 4, Section 4.4) and the top-left k x k
// block of H^-1 (eq. equ:index, Section 4.5) on the scaled integer factor.
//
// Scaled form: with Q = W - G, G = max_{m<k} s_m + 64,
//   x_mm = 2^(Q - h_m),   x_rm = rnd( -(sum_{i=m}^{r-1} b_ri x_im) / 2^h_r )  (r > m),
// and with the per-pivot reciprocals w_r = rnd(2^(2 h_r + P) / d_r):
//   M_ab = sum_{r >= max(a,b)} x_ra x_rb w_r   (exact),
//   (H^-1)_ab = M_ab 2^(W - 2Q - P - s_a - s_b).
// The block is brought to one exponent and rounded once to P-2 bits.
//
// The sums for row r are accumulated in a 2P-bit two's complement accumulator
// ACC[r][m] = -sum_i b_ri x_im, by the same exact update kernel that does the
// Schur complement (A[r][c] -= sum_i b_ri u_ci with u_ci := x_im); rows are
// finished in blocks of 16, each finished block updating all later rows.
#include "hl_kernels.hpp"

namespace hl {

__device__ __forceinline__ int q_of(const i32* s, int k, int W) {
  int mx = s[0];
  for (int m = 1; m < k; ++m) mx = s[m] > mx ? s[m] : mx;
  return W - (mx + 64);
}

constexpr int TRSM_THREADS = 256;
// LDS words of the carry-chain table for nw limbs (as wg_resolve needs)
__host__ __device__ constexpr int trsm_rip_words(int nw) { return 2 * ((nw + WAVE - 1) / WAVE) + 4; }

// Finish row r of X: one workgroup of TRSM_THREADS per column m, the carry
// chains resolved by the whole workgroup.
__device__ void trsm_row_body(const TrsmRowArgs& a, int m) {
  const u32* __restrict__ ACC = a.ACC;
  const Dims dm = a.dm;
  const int r = a.r;
  const i32* __restrict__ s = a.s;
  const i32* __restrict__ h = a.h;
  u32* __restrict__ X = a.X;
  DevStatus* st = a.st;
  if (has_error(st) || m >= dm.k) return;
  const int nl = dm.nl, nw = dm.nw;
  u32* xo = X + ((size_t)r * dm.k + m) * nl;
  if (r < m) {
    for (int l = threadIdx.x; l < nl; l += blockDim.x) xo[l] = 0;
    return;
  }
  if (r == m) {
    const int Q = q_of(s, dm.k, dm.W);
    const int e = Q - h[m];
    if (e < 0 || e > dm.P - 2) {
      if (threadIdx.x == 0) set_status(st, HL_EOVERFLOW, r);
      return;
    }
    for (int l = threadIdx.x; l < nl; l += blockDim.x) xo[l] = (l == (e >> 5)) ? (1u << (e & 31)) : 0u;
    return;
  }
  extern __shared__ u32 lds[];
  u32* As = lds;           // nw + 4
  u32* Xs = As + nw + 4;   // nl + 4
  u32* rip = Xs + nl + 4;  // trsm_rip_words(nw)
  const u32* src = ACC + (size_t)(r >> 5) * tile_words(nw);
  for (int l = threadIdx.x; l < nw; l += blockDim.x) As[l] = src[in_tile(r, m, l)];
  __syncthreads();
  // every thread reads the sign before the negation's first write (which
  // follows two of its barriers)
  const bool neg = (As[nw - 1] >> 31) != 0;
  if (neg) wg_neg(As, nw, rip);
  const int hr = h[r];
  if (hr > 0) {
    const int pos = (hr - 1) >> 5;
    const u32 v = 1u << ((hr - 1) & 31);
    wg_resolve(nw, [=](int p) -> u64 { return (u64)As[p] + (p == pos ? v : 0u); }, As, rip);
  }
  wg_shift_right(As, nw, hr, Xs, nl + 1);
  if (Xs[nl] != 0 || Xs[nl - 1] >= 0x60000000u) {
    if (threadIdx.x == 0) set_status(st, HL_EOVERFLOW, r);
    return;
  }
  if (neg) wg_neg(Xs, nl, rip);
  for (int l = threadIdx.x; l < nl; l += blockDim.x) xo[l] = Xs[l];
}

__global__ __launch_bounds__(TRSM_THREADS) void k_trsm_row(TrsmRowArgs a) { trsm_row_body(a, blockIdx.x); }

// batch: blockIdx.y is the instance
__global__ __launch_bounds__(TRSM_THREADS) void k_trsm_row_b(const TrsmRowArgs* __restrict__ tab) {
  trsm_row_body(tab[blockIdx.y], blockIdx.x);
}

// ---------------------------------------------------------------------------
// Block partial sums: pair p = (a, b), a <= b, rows [ch*R, ch*R + R) with r >= b.
// part[p][ch] = sum x_ra x_rb w_r, two's complement over ns limbs.
__global__ __launch_bounds__(64) void k_block_part(const u32* __restrict__ X, Dims dm,
                                                   const u32* __restrict__ omega, int ostride,
                                                   int rows_per_chunk, u32* __restrict__ part, int ns,
                                                   int nchunks, DevStatus* st) {
  if (has_error(st)) return;
  const int p = blockIdx.x, ch = blockIdx.y;
  // p -> (a, b) with a <= b: p = b (b + 1) / 2 + a
  int b = 0;
  while ((b + 1) * (b + 2) / 2 <= p) ++b;
  const int a = p - b * (b + 1) / 2;
  const int nl = dm.nl, k = dm.k;
  u32* acc = part + ((size_t)p * nchunks + ch) * ns;
  for (int l = lane_id(); l < ns; l += WAVE) acc[l] = 0;
  extern __shared__ u32 lds[];
  u32* xa = lds;               // nl
  u32* xb = xa + nl;           // nl
  u32* om = xb + nl;           // nl + 2
  u32* p1 = om + nl + 2;       // 2 nl + 2
  u32* p2 = p1 + 2 * nl + 2;   // 3 nl + 4
  const int r0 = max(ch * rows_per_chunk, b), r1 = min(ch * rows_per_chunk + rows_per_chunk, dm.N);
  for (int r = r0; r < r1; ++r) {
    __syncthreads();
    const u32* pa = X + ((size_t)r * k + a) * nl;
    const u32* pb = X + ((size_t)r * k + b) * nl;
    const u32* po = omega + (size_t)r * ostride;
    for (int l = lane_id(); l < nl; l += WAVE) {
      xa[l] = pa[l];
      xb[l] = pb[l];
    }
    for (int l = lane_id(); l < nl + 2; l += WAVE) om[l] = po[l];
    __syncthreads();
    const bool na = (xa[nl - 1] >> 31) != 0, nb = (xb[nl - 1] >> 31) != 0;
    if (na) w_neg(xa, nl);
    if (nb) w_neg(xb, nl);
    __syncthreads();
    w_mul(xa, nl, xb, nl, p1, 2 * nl);
    __syncthreads();
    w_mul(p1, 2 * nl, om, nl + 1, p2, 3 * nl + 1);
    __syncthreads();
    if (na != nb) {
      // acc -= p2 : acc + ~p2 + 1 over ns limbs (p2 zero-extended)
      u32 carry = 1;
      for (int base = 0; base < ns; base += WAVE) {
        const int q = base + lane_id();
        u64 v = 0;
        if (q < ns) v = (u64)acc[q] + (u64)(~(q < 3 * nl + 1 ? p2[q] : 0u));
        const u32 limb = w_resolve(v, carry);
        if (q < ns) acc[q] = limb;
      }
    } else {
      w_add(acc, ns, p2, 3 * nl + 1, acc, ns);
    }
  }
}

// Sum of the partials of pair p, shifted to the common scale 2^(2 s* - s_a - s_b).
__global__ __launch_bounds__(64) void k_block_reduce(const u32* __restrict__ part, int ns, int nchunks,
                                                     const i32* __restrict__ s, Dims dm,
                                                     u32* __restrict__ msum, int nm, DevStatus* st) {
  if (has_error(st)) return;
  const int p = blockIdx.x;
  int b = 0;
  while ((b + 1) * (b + 2) / 2 <= p) ++b;
  const int a = p - b * (b + 1) / 2;
  extern __shared__ u32 lds[];
  u32* acc = lds;  // nm limbs
  for (int l = lane_id(); l < nm; l += WAVE) acc[l] = 0;
  __syncthreads();
  for (int ch = 0; ch < nchunks; ++ch) {
    w_add(acc, ns, part + ((size_t)p * nchunks + ch) * ns, ns, acc, ns);
    __syncthreads();
  }
  // sign-extend the ns-limb sum to nm limbs
  const u32 ext = (acc[ns - 1] >> 31) ? 0xffffffffu : 0u;
  for (int l = ns + lane_id(); l < nm; l += WAVE) acc[l] = ext;
  __syncthreads();
  int smax = s[0];
  for (int m = 1; m < dm.k; ++m) smax = s[m] > smax ? s[m] : smax;
  const long sh = 2L * smax - s[a] - s[b];
  if (sh < 0 || sh > 32L * (nm - ns) - 32) {
    if (lane_id() == 0) set_status(st, HL_EOVERFLOW, p);
    return;
  }
  u32* out = msum + (size_t)p * nm;
  for (int j = lane_id(); j < nm; j += WAVE) out[j] = limb_shl(acc, nm, sh, j);
}

// Common exponent and rounding to P-2 bits; one wave.
__global__ __launch_bounds__(64) void k_block_final(const u32* __restrict__ msum, int nm, Dims dm,
                                                    const i32* __restrict__ s, u32* __restrict__ blk,
                                                    i64* __restrict__ blk_exp, DevStatus* st) {
  if (has_error(st)) return;
  extern __shared__ u32 lds[];
  u32* t = lds;  // nm + 4
  const int k = dm.k, nl = dm.nl, npairs = k * (k + 1) / 2;
  int maxbl = 0;
  for (int p = 0; p < npairs; ++p) {
    const u32* m = msum + (size_t)p * nm;
    __syncthreads();
    for (int l = lane_id(); l < nm; l += WAVE) t[l] = m[l];
    __syncthreads();
    if (t[nm - 1] >> 31) w_neg(t, nm);
    __syncthreads();
    const int bl = w_bitlen(t, nm);
    maxbl = bl > maxbl ? bl : maxbl;
  }
  const int tau = maxbl - (dm.P - 2) > 0 ? maxbl - (dm.P - 2) : 0;
  int smax = s[0];
  for (int m = 1; m < k; ++m) smax = s[m] > smax ? s[m] : smax;
  const int Q = dm.W - (smax + 64);
  if (lane_id() == 0) blk_exp[0] = (i64)dm.W - 2L * Q - dm.P - 2L * smax + tau;
  u32* o = t + nm + 4;  // nl + 4
  for (int p = 0; p < npairs; ++p) {
    int b = 0;
    while ((b + 1) * (b + 2) / 2 <= p) ++b;
    const int a = p - b * (b + 1) / 2;
    const u32* m = msum + (size_t)p * nm;
    __syncthreads();
    for (int l = lane_id(); l < nm; l += WAVE) t[l] = m[l];
    __syncthreads();
    const bool neg = (t[nm - 1] >> 31) != 0;
    if (neg) w_neg(t, nm);
    __syncthreads();
    if (tau > 0) w_add_word(t, nm, (tau - 1) >> 5, 1u << ((tau - 1) & 31));
    __syncthreads();
    w_shift_right(t, nm, tau, o, nl);
    __syncthreads();
    if (neg) w_neg(o, nl);
    __syncthreads();
    for (int l = lane_id(); l < nl; l += WAVE) {
      blk[((size_t)a * k + b) * nl + l] = o[l];
      blk[((size_t)b * k + a) * nl + l] = o[l];
    }
  }
}

// ---------------------------------------------------------------------------
// MFMA form of the block sums: M_ab = sum_r (x_rb w_r) x_ra.  k_block_y forms
// y_rb = x_rb w_r (one workgroup per (r, b), both factors in LDS); the sum over
// r is a Toeplitz-form MFMA GEMM of y against x (k rows b, k columns a, rank r),
// and k_block_gather moves M_ab (a <= b) into the pair layout of k_block_reduce.
constexpr int BY_THREADS = 256;
size_t block_y_lds_bytes(int nl) { return (size_t)(nl + (nl + 1) + (2 * nl + 1) + 3 * (2 * nl + 1) + 8) * 4; }

__global__ __launch_bounds__(BY_THREADS) void k_block_y(const u32* __restrict__ X, Dims dm,
                                                         const u32* __restrict__ omega, int ostride,
                                                         u32* __restrict__ Y, int ny, DevStatus* st) {
  if (has_error(st)) return;
  const int r = blockIdx.x, b = blockIdx.y;
  const int nl = dm.nl, k = dm.k;
  u32* yo = Y + ((size_t)b * dm.NT + r) * ny;
  if (r >= dm.N) {
    for (int l = threadIdx.x; l < ny; l += blockDim.x) yo[l] = 0;
    return;
  }
  extern __shared__ u32 lds[];
  u32* xs = lds;                 // nl
  u32* om = xs + nl;             // nl + 1
  u32* pr = om + nl + 1;         // 2 nl + 1
  u32* cb = pr + 2 * nl + 1;     // 3 (2 nl + 1)
  int* flag = (int*)(cb + 3 * (2 * nl + 1));
  const u32* px = X + ((size_t)r * k + b) * nl;
  const u32* po = omega + (size_t)r * ostride;
  for (int l = threadIdx.x; l < nl; l += blockDim.x) xs[l] = px[l];
  for (int l = threadIdx.x; l < nl + 1; l += blockDim.x) om[l] = po[l];
  __syncthreads();
  if (wave_id() == 0) {
    const bool neg = (xs[nl - 1] >> 31) != 0;
    if (neg) w_neg(xs, nl);
    if (lane_id() == 0) flag[0] = neg ? 1 : 0;
  }
  __syncthreads();
  const bool neg = flag[0] != 0;
  g_mul(xs, nl, om, nl + 1, pr, 2 * nl + 1, cb);
  if (wave_id() == 0 && neg) w_neg(pr, 2 * nl + 1);
  __syncthreads();
  const u32 ext = neg && !w_is_zero(pr, 2 * nl + 1) ? 0xffffffffu : 0u;
  for (int l = threadIdx.x; l < ny; l += blockDim.x) yo[l] = l < 2 * nl + 1 ? pr[l] : ext;
}

// part[p][0] = M_(b, a) (nm limbs, sign-extended to ns), p = b (b + 1) / 2 + a;
// with M2 (the sums over the other half of the rows r), M_(b, a) + M2_(b, a)
// (two's complement over nm limbs, which hold the exact sum)
__global__ __launch_bounds__(64) void k_block_gather(const u32* __restrict__ M, const u32* __restrict__ M2, int nm,
                                                     Dims dm, u32* __restrict__ part, int ns, DevStatus* st) {
  if (has_error(st)) return;
  const int p = blockIdx.x;
  int b = 0;
  while ((b + 1) * (b + 2) / 2 <= p) ++b;
  const int a = p - b * (b + 1) / 2;
  const u32* m = M + ((size_t)b * dm.k + a) * nm;
  u32* o = part + (size_t)p * ns;
  if (M2) {
    w_add(m, nm, M2 + ((size_t)b * dm.k + a) * nm, nm, o, nm);
    wsync();
    m = o;
  }
  const u32 ext = (m[nm - 1] >> 31) ? 0xffffffffu : 0u;
  for (int l = lane_id(); l < ns; l += WAVE) o[l] = l < nm ? m[l] : ext;
}

// ---------------------------------------------------------------------------
hipError_t launch_trsm_row(const u32* ACC, const Dims& dm, int r, const i32* s, const i32* h, u32* X,
                           DevStatus* st, hipStream_t stream) {
  const size_t lds = (size_t)(dm.nw + 4 + dm.nl + 4 + trsm_rip_words(dm.nw)) * 4;
  const TrsmRowArgs a{ACC, dm, r, s, h, X, st};
  hipLaunchKernelGGL(k_trsm_row, dim3(dm.k), dim3(TRSM_THREADS), lds, stream, a);
  return hipGetLastError();
}

hipError_t launch_trsm_row_batch(const TrsmRowArgs* tab, int count, int k_max, int nl_max, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const size_t lds = (size_t)(2 * nl_max + 4 + nl_max + 4 + trsm_rip_words(2 * nl_max)) * 4;
  hipLaunchKernelGGL(k_trsm_row_b, dim3(k_max, count), dim3(TRSM_THREADS), lds, stream, tab);
  return hipGetLastError();
}

hipError_t launch_block(const u32* X, const Dims& dm, const u32* omega, int ostride, const i32* s,
                        u32* part, int ns, int nchunks, int rows_per_chunk, u32* msum, int nm, u32* blk,
                        i64* blk_exp, DevStatus* st, hipStream_t stream) {
  const int npairs = dm.k * (dm.k + 1) / 2;
  const size_t lds1 = (size_t)(2 * dm.nl + dm.nl + 2 + 2 * dm.nl + 2 + 3 * dm.nl + 4) * 4;
  hipLaunchKernelGGL(k_block_part, dim3(npairs, nchunks), dim3(64), lds1, stream, X, dm, omega, ostride,
                     rows_per_chunk, part, ns, nchunks, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_block_sums(dm, s, part, ns, nchunks, msum, nm, blk, blk_exp, st, stream);
}

static hipError_t allow_lds_solve(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_block_y(const u32* X, const Dims& dm, const u32* omega, int ostride, u32* Y, int ny,
                          DevStatus* st, hipStream_t stream) {
  if (ny < 2 * dm.nl + 1) return hipErrorInvalidValue;
  const size_t lds = block_y_lds_bytes(dm.nl);
  hipError_t e = allow_lds_solve((const void*)k_block_y, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_block_y, dim3(dm.NT, dm.k), dim3(BY_THREADS), lds, stream, X, dm, omega, ostride, Y, ny, st);
  return hipGetLastError();
}

hipError_t launch_block_gather(const u32* M, const u32* M2, int nm, const Dims& dm, u32* part, int ns, DevStatus* st,
                               hipStream_t stream) {
  if (ns < nm) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_block_gather, dim3(dm.k * (dm.k + 1) / 2), dim3(64), 0, stream, M, M2, nm, dm, part, ns, st);
  return hipGetLastError();
}

// sum of the nchunks partials of each pair, common exponent, rounding
hipError_t launch_block_sums(const Dims& dm, const i32* s, const u32* part, int ns, int nchunks, u32* msum, int nm,
                             u32* blk, i64* blk_exp, DevStatus* st, hipStream_t stream) {
  const int npairs = dm.k * (dm.k + 1) / 2;
  hipError_t e;
  hipLaunchKernelGGL(k_block_reduce, dim3(npairs), dim3(64), (size_t)nm * 4, stream, part, ns, nchunks, s,
                     dm, msum, nm, st);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_block_final, dim3(1), dim3(64), (size_t)(nm + 4 + dm.nl + 4) * 4, stream, msum, nm,
                     dm, s, blk, blk_exp, st);
  return hipGetLastError();
}

}  // namespace hl
