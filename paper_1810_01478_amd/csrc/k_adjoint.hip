// Adjoint of lambda_1 with respect to the moments, contracted with a moment
// direction dmu (d mu / d beta for the derivative in beta).
//
// First-order perturbation of the largest eigenvalue of the block M of H^-1
// (Sections 4.2 and 4.5): with y the eigenvector of M for lambda_max,
//   d lambda_1 = v^T dH v / (y^T y),   v = lambda_1 H^-1 E y,
// and dH_ij = dmu_{i+j}, so mubar_m = sum_{i+j=m} v_i v_j is d lambda_1 / d mu_m.
//
// Scaled form.  The factorisation holds A~ = 2^W S^-1 H S^-1 (S = diag 2^s) as
// A~ = B Delta B^T with B_ri = b_ri (r > i), B_ii = 2^h_i, Delta_i = d_i 2^-2h_i,
// and X = 2^Q B^-1 E (the first k columns, from the triangular solve).  Then
//   z := A~^-1 S^-1 E y = B^-T Delta^-1 B^-1 S^-1 E y,
//   v = lambda_1 2^W S^-1 z,   v^T dH v = lambda_1^2 2^W z^T dA~ z,
// where dA~_ij = dmu_{i+j} 2^(W - s_i - s_j).  In integers:
//   Y_m  = rnd(y_m 2^(P-3)),  Yc_m = rnd(Y_m / 2^(s_m - s0)),  s0 = min_{m<k} s_m
//   T_r  = sum_m x_rm Yc_m                                       (exact)
//   G_r  = rnd(T_r w_r 2^eG),  eG = F - Q - s0 - 2P + 3,  w_r = rnd(2^(2h_r+P)/d_r)
//   z_i  = rnd((G_i - sum_{r>i} b_ri z_r) / 2^h_i),  i = N-1 .. 0  (B^T z = G)
//   da_ij = rnd(dmu_{i+j} 2^(W' - s_i - s_j)),  W' the largest value keeping
//           every |da_ij| below 2^(2P-3)
//   Tot  = sum_i z_i sum_j da_ij z_j                              (exact)
//   d lambda_1 = lambda_1^2 2^(2W - W' - 2F + 2P - 6) Tot / sum_m Y_m^2.
// F (the binary point of z) is chosen by the host so that |z_i| stays below
// 2^(P-3); a z outside 3 2^(P-3) is reported as EOVERFLOW.
#include "hl_kernels.hpp"
#include "hl_host.hpp"

namespace hl {

// value of the signed number x (two's complement, n limbs) rounded to nearest,
// ties away from zero, after a right shift by sh >= 0 (sh < 0: exact left shift);
// result into dst (nd limbs, two's complement, modulo 2^(32 nd)).  tmp: n + 2 words.
__device__ void w_round_shift(const u32* x, int n, long sh, u32* dst, int nd, u32* tmp) {
  const bool neg = (x[n - 1] >> 31) != 0;
  w_copy(x, tmp, n);
  wsync();
  if (neg) w_neg(tmp, n);
  wsync();
  if (sh > 0) w_add_word(tmp, n, (int)((sh - 1) >> 5), 1u << ((sh - 1) & 31));
  wsync();
  for (int j = lane_id(); j < nd; j += WAVE) {
    const u32 v = sh >= 0 ? limb_shr(tmp, n, sh, j) : limb_shl(tmp, n, -sh, j);
    dst[j] = v;
  }
  wsync();
  if (neg) w_neg(dst, nd);
  wsync();
}

// acc (na limbs, two's complement) += (neg ? -1 : 1) * a * b, a and b unsigned
// (na, nb limbs); the product is formed column chunk by column chunk and added
// on the fly, so no product buffer is needed.  acc must be in LDS or global
// memory private to the wave.
__device__ void w_mac(u32* acc, int nacc, const u32* a, int na, const u32* b, int nb, bool neg) {
  const int nch = (nacc + WAVE - 1) / WAVE;
  u32 carry = neg ? 1u : 0u;
  const int nprod = (na + nb + WAVE - 1) / WAVE;
  const int l = lane_id();
  w_mul_stream(a, na, b, nb, nprod < nch ? nprod : nch, [&](int ch, u32 limb) {
    const int p = ch * WAVE + l;
    u64 v = 0;
    if (p < nacc) v = (u64)acc[p] + (u64)(neg ? ~limb : limb);
    const u32 out = w_resolve(v, carry);
    if (p < nacc) acc[p] = out;
  });
  // limbs above the product: add 0 (or ~0 for the negated product)
  for (int ch = nprod; ch < nch; ++ch) {
    if (!neg && carry == 0) break;
    const int p = ch * WAVE + l;
    u64 v = 0;
    if (p < nacc) v = (u64)acc[p] + (u64)(neg ? 0xffffffffu : 0u);
    const u32 out = w_resolve(v, carry);
    if (p < nacc) acc[p] = out;
  }
  wsync();
}

// ---------------------------------------------------------------------------
// Y_m, Yc_m and sum_m Y_m^2 from the eigen-step's vector (multiprecision floats
// with exponent <= 0).  One workgroup; wave w takes m = w, w + nwaves, ...
__global__ __launch_bounds__(256) void k_adj_y(const int* __restrict__ yhdr, const u32* __restrict__ ymant, int NWM,
                                               Dims dm, const i32* __restrict__ s, u32* __restrict__ Y,
                                               u32* __restrict__ Yc, u32* __restrict__ ysq, DevStatus* st) {
  if (has_error(st)) return;
  const int nl = dm.nl, k = dm.k, P = dm.P;
  const int w = wave_id(), nwv = blockDim.x / WAVE;
  extern __shared__ u32 lds[];
  u32* tmp = lds + (size_t)w * (2 * NWM + 2 * nl + 16);
  u32* mag = tmp + NWM + 4;
  int s0 = s[0];
  for (int m = 1; m < k; ++m) s0 = s[m] < s0 ? s[m] : s0;
  for (int m = w; m < k; m += nwv) {
    u32* ym = Y + (size_t)m * nl;
    if (k == 1) {
      // a 1 x 1 block: the eigenvector is 1
      for (int j = lane_id(); j < nl; j += WAVE) ym[j] = (j == (P - 3) >> 5) ? (1u << ((P - 3) & 31)) : 0u;
    } else {
      const int sign = yhdr[2 * m], ex = yhdr[2 * m + 1];
      if (sign == 2) {
        for (int j = lane_id(); j < nl; j += WAVE) ym[j] = 0;
      } else {
        // y = (M / 2^(32 NWM)) 2^ex; Y = rnd(y 2^(P-3)) = rnd(M / 2^(32 NWM - ex - P + 3))
        const long sh = 32L * NWM - ex - (P - 3);
        const u32* M = ymant + (size_t)m * NWM;
        w_copy(M, tmp, NWM);
        if (lane_id() == 0) tmp[NWM] = 0;
        wsync();
        if (sh > 0) w_add_word(tmp, NWM + 1, (int)((sh - 1) >> 5), 1u << ((sh - 1) & 31));
        wsync();
        for (int j = lane_id(); j < nl; j += WAVE) mag[j] = limb_shr(tmp, NWM + 1, sh, j);
        wsync();
        if (sign) w_neg(mag, nl);
        wsync();
        w_copy(mag, ym, nl);
      }
    }
    wsync();
    // Yc_m = rnd(Y_m / 2^(s_m - s0))
    w_round_shift(ym, nl, (long)s[m] - s0, Yc + (size_t)m * nl, nl, tmp);
  }
  __syncthreads();
  if (w == 0) {
    // sum_m Y_m^2 (nonnegative, 2 nl + 2 limbs)
    u32* acc = tmp;
    mag = tmp + 2 * nl + 4;
    w_fill(acc, 2 * nl + 2, 0u);
    wsync();
    for (int m = 0; m < k; ++m) {
      w_copy(Y + (size_t)m * nl, mag, nl);
      wsync();
      if (mag[nl - 1] >> 31) w_neg(mag, nl);
      wsync();
      w_mac(acc, 2 * nl + 2, mag, nl, mag, nl, false);
    }
    w_copy(acc, ysq, 2 * nl + 2);
  }
}

// G_r = rnd(T_r w_r 2^eG), T_r = sum_m x_rm Yc_m, into the accumulator entry
// (r, 0) of the rectangular tile storage.  One wave per row.
__global__ __launch_bounds__(64) void k_adj_g(const u32* __restrict__ X, const u32* __restrict__ Yc,
                                              const u32* __restrict__ omega, int ostride, Dims dm, long eG,
                                              u32* __restrict__ ACC, DevStatus* st) {
  if (has_error(st)) return;
  const int r = blockIdx.x;
  const int nl = dm.nl, nw = dm.nw, k = dm.k;
  extern __shared__ u32 lds[];
  const int nt = 2 * nl + 2;       // T: 2P + log2 k bits
  const int np = nt + nl + 2;      // T w
  u32* T = lds;                    // nt
  u32* xa = T + nt;                // nl
  u32* ya = xa + nl;               // nl
  u32* om = ya + nl;               // nl + 2
  u32* pr = om + nl + 2;           // np (and its rounded shift)
  u32* tmp = pr + np;              // np + 2
  u32* g = tmp + np + 2;           // nw
  w_fill(T, nt, 0u);
  wsync();
  for (int m = 0; m < k && m <= r; ++m) {
    w_copy(X + ((size_t)r * k + m) * nl, xa, nl);
    w_copy(Yc + (size_t)m * nl, ya, nl);
    wsync();
    const bool nx = (xa[nl - 1] >> 31) != 0, ny = (ya[nl - 1] >> 31) != 0;
    if (nx) w_neg(xa, nl);
    if (ny) w_neg(ya, nl);
    wsync();
    w_mac(T, nt, xa, nl, ya, nl, nx != ny);
  }
  // |T| w, then the rounded shift, then the sign
  const bool nT = (T[nt - 1] >> 31) != 0;
  if (nT) w_neg(T, nt);
  for (int j = lane_id(); j < nl + 2; j += WAVE) om[j] = j < ostride ? omega[(size_t)r * ostride + j] : 0u;
  wsync();
  w_fill(pr, np, 0u);
  wsync();
  w_mac(pr, np, T, nt, om, nl + 2, false);
  w_round_shift(pr, np, -eG, g, nw, tmp);
  if (nT) w_neg(g, nw);
  wsync();
  u32* dst = ACC + (size_t)(r >> 5) * tile_words(nw);
  for (int l = lane_id(); l < nw; l += WAVE) dst[in_tile(r, 0, l)] = g[l];
}

// z_i = rnd(ACC_i / 2^h_i), checked against 3 2^(P-3).  One wave.
// z_i = rnd(acc_i / 2^h_i) of one row, by one workgroup (the carry chains
// resolved by all its waves); same value as w_round_shift.
constexpr int ADJ_ROW_THREADS = 256;
__host__ __device__ constexpr int adj_rip_words(int nw) { return 2 * ((nw + WAVE - 1) / WAVE) + 4; }
__global__ __launch_bounds__(ADJ_ROW_THREADS) void k_adj_row(const u32* __restrict__ ACC, Dims dm, int i,
                                                             const i32* __restrict__ h, u32* __restrict__ Z,
                                                             DevStatus* st) {
  if (has_error(st)) return;
  const int nl = dm.nl, nw = dm.nw;
  extern __shared__ u32 lds[];
  u32* a = lds;             // nw + 2
  u32* z = a + nw + 2;      // nl + 2
  u32* rip = z + nl + 2;    // adj_rip_words(nw)
  const u32* src = ACC + (size_t)(i >> 5) * tile_words(nw);
  for (int l = threadIdx.x; l < nw; l += blockDim.x) a[l] = src[in_tile(i, 0, l)];
  __syncthreads();
  // |a| rounded to nearest (ties away from zero) at bit sh, then the sign back
  const bool neg = (a[nw - 1] >> 31) != 0;
  if (neg) wg_neg(a, nw, rip);
  const long sh = h[i];
  if (sh > 0) {
    const int pos = (int)((sh - 1) >> 5);
    const u32 v = 1u << ((sh - 1) & 31);
    wg_resolve(nw, [=](int p) -> u64 { return (u64)a[p] + (p == pos ? v : 0u); }, a, rip);
  }
  wg_shift_right(a, nw, sh, z, nl + 1);
  if (neg) wg_neg(z, nl + 1, rip);
  // |z| < 3 2^(P-3): the top limb of the sign-extended value is 0 or ~0 and
  // limb nl-1 lies within the bound
  const u32 top = z[nl], t1 = z[nl - 1];
  const bool ok = (top == 0 && t1 < 0x60000000u) || (top == 0xffffffffu && t1 > 0xa0000000u);
  if (!ok) {
    if (threadIdx.x == 0) set_status(st, HL_EOVERFLOW, i);
    return;
  }
  for (int l = threadIdx.x; l < nl; l += blockDim.x) Z[(size_t)i * nl + l] = z[l];
}

// W' = min_m (2P - 3 - bitlen(dmu_m) + min_{i+j=m} (s_i + s_j)) over nonzero dmu_m.
__global__ __launch_bounds__(256) void k_adj_wprime(const u32* __restrict__ dmu, const i64* __restrict__ dexp, int w,
                                                    Dims dm, const i32* __restrict__ s, i64* __restrict__ out) {
  __shared__ long red[256];
  const int N = dm.N;
  long best = LONG_MAX;
  for (int m = threadIdx.x; m < 2 * N - 1; m += blockDim.x) {
    const u32* M = dmu + (size_t)m * w;
    int top = w - 1;
    while (top >= 0 && M[top] == 0) --top;
    if (top < 0) continue;
    const long bl = (long)top * 32 + (32 - __clz((int)M[top])) + dexp[m];
    int ms = INT_MAX;
    const int lo = m - (N - 1) > 0 ? m - (N - 1) : 0, hi = m < N - 1 ? m : N - 1;
    for (int i = lo; i <= hi; ++i) ms = s[i] + s[m - i] < ms ? s[i] + s[m - i] : ms;
    const long v = 2L * dm.P - 3 - bl + ms;
    best = v < best ? v : best;
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o && red[threadIdx.x + o] < red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// part_i = z_i sum_j da_ij z_j (two's complement, ns = 4 nl + 4 limbs).
// One workgroup of up to ADJ_WAVES waves per row i; wave w takes j = w,
// w + nwaves, ...
constexpr int ADJ_WAVES = 4;
__global__ __launch_bounds__(ADJ_WAVES * 64) void k_adj_contract(
    const u32* __restrict__ dmu, const i64* __restrict__ dexp, const int* __restrict__ dneg, int w, Dims dm,
    const i32* __restrict__ s, const i64* __restrict__ wprime, const u32* __restrict__ Z, u32* __restrict__ part,
    DevStatus* st) {
  if (has_error(st)) return;
  const int i = blockIdx.x;
  const int N = dm.N, nl = dm.nl, nw = dm.nw;
  const int nr = 3 * nl + 4;   // sum_j da_ij z_j
  const int ns = 4 * nl + 4;   // z_i times that
  const int wv = wave_id(), nwv = blockDim.x / WAVE;
  extern __shared__ u32 lds[];
  const int per = nw + 4 + nl + 2 + nr;
  u32* da = lds + (size_t)wv * per;  // nw + 4 (magnitude, then rounded)
  u32* zj = da + nw + 4;              // nl + 2
  u32* acc = zj + nl + 2;             // nr
  const long Wp = wprime[0];
  w_fill(acc, nr, 0u);
  wsync();
  for (int j = wv; j < N; j += nwv) {
    const int m = i + j;
    const u32* M = dmu + (size_t)m * w;
    // |da_ij| = rnd(|dmu_m| 2^(e_m + W' - s_i - s_j)) over nw limbs
    const long sh = dexp[m] + Wp - s[i] - s[j];
    u32 cy = 0;
    if (sh < 0) cy = get_bit(M, w, -sh - 1);
    {
      u32 carry = cy;
      for (int base = 0; base < nw; base += WAVE) {
        const int p = base + lane_id();
        u64 v = 0;
        if (p < nw) v = sh >= 0 ? limb_shl(M, w, sh, p) : limb_shr(M, w, -sh, p);
        const u32 limb = w_resolve(v, carry);
        if (p < nw) da[p] = limb;
      }
    }
    w_copy(Z + (size_t)j * nl, zj, nl);
    wsync();
    const bool nz = (zj[nl - 1] >> 31) != 0;
    if (nz) w_neg(zj, nl);
    wsync();
    w_mac(acc, nr, da, nw, zj, nl, (dneg[m] != 0) != nz);
  }
  __syncthreads();
  if (wv == 0) {
    // R_i = sum of the waves' accumulators
    for (int q = 1; q < nwv; ++q) {
      const u32* other = lds + (size_t)q * per + nw + 4 + nl + 2;
      w_add(acc, nr, other, nr, acc, nr);
      wsync();
    }
    // part_i = z_i R_i
    const bool nR = (acc[nr - 1] >> 31) != 0;
    if (nR) w_neg(acc, nr);
    w_copy(Z + (size_t)i * nl, zj, nl);
    wsync();
    const bool nz = (zj[nl - 1] >> 31) != 0;
    if (nz) w_neg(zj, nl);
    wsync();
    u32* out = part + (size_t)i * ns;
    for (int p = lane_id(); p < ns; p += WAVE) out[p] = 0;
    wsync();
    w_mac(out, ns, acc, nr, zj, nl, nR != nz);
  }
}

// MFMA form of the contraction: the sums R_i = sum_j da_ij z_j run as
// Toeplitz-form int8 GEMMs of rank 16 over j.  k_adj_da writes da_ij for the 16
// columns j0 .. j0+15 of a launch as two's complement (nw limbs, da[p][i]);
// k_adj_part then forms part_i = z_i R_i.
__global__ __launch_bounds__(64) void k_adj_da(const u32* __restrict__ dmu, const i64* __restrict__ dexp,
                                               const int* __restrict__ dneg, int w, Dims dm,
                                               const i32* __restrict__ s, const i64* __restrict__ wprime, int j0,
                                               u32* __restrict__ DA, int lda, DevStatus* st) {
  if (has_error(st)) return;
  const int i = blockIdx.x, p = blockIdx.y, j = j0 + p;
  const int nw = dm.nw, m = i + j;
  u32* da = DA + ((size_t)p * dm.N + i) * lda;
  const u32* M = dmu + (size_t)m * w;
  // |da_ij| = rnd(|dmu_m| 2^(e_m + W' - s_i - s_j)) over nw limbs, as k_adj_contract
  const long sh = dexp[m] + wprime[0] - s[i] - s[j];
  u32 carry = sh < 0 ? get_bit(M, w, -sh - 1) : 0u;
  for (int base = 0; base < nw; base += WAVE) {
    const int q = base + lane_id();
    u64 v = 0;
    if (q < nw) v = sh >= 0 ? limb_shl(M, w, sh, q) : limb_shr(M, w, -sh, q);
    const u32 limb = w_resolve(v, carry);
    if (q < nw) da[q] = limb;
  }
  wsync();
  if (dneg[m]) w_neg(da, nw);
}

__global__ __launch_bounds__(64) void k_adj_part(const u32* __restrict__ R, int nr, const u32* __restrict__ Z, Dims dm,
                                                 u32* __restrict__ part, DevStatus* st) {
  if (has_error(st)) return;
  const int i = blockIdx.x, nl = dm.nl;
  const int ns = 4 * nl + 4;
  extern __shared__ u32 lds[];
  u32* acc = lds;       // nr
  u32* zj = acc + nr;   // nl
  w_copy(R + (size_t)i * nr, acc, nr);
  w_copy(Z + (size_t)i * nl, zj, nl);
  wsync();
  const bool nR = (acc[nr - 1] >> 31) != 0, nz = (zj[nl - 1] >> 31) != 0;
  if (nR) w_neg(acc, nr);
  if (nz) w_neg(zj, nl);
  u32* out = part + (size_t)i * ns;
  for (int q = lane_id(); q < ns; q += WAVE) out[q] = 0;
  wsync();
  w_mac(out, ns, acc, nr, zj, nl, nR != nz);
}

// column sums of the parts (each limb position summed over rows as u64), then
// one wave resolves the carries: the sum of two's complement numbers mod 2^(32 ns)
__global__ __launch_bounds__(256) void k_adj_colsum(const u32* __restrict__ part, int N, int ns,
                                                    unsigned long long* __restrict__ col) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  unsigned long long acc = 0;
  for (int i = 0; i < N; ++i) acc += part[(size_t)i * ns + p];
  col[p] = acc;
}

__global__ __launch_bounds__(64) void k_adj_resolve(const unsigned long long* __restrict__ col, int ns,
                                                    u32* __restrict__ tot) {
  u32 carry = 0;
  u32 spill = 0;  // high word of the previous chunk's last column
  for (int base = 0; base < ns; base += WAVE) {
    const int p = base + lane_id();
    const unsigned long long c = p < ns ? col[p] : 0ull;
    // value at position p: low word of col[p] + high word of col[p-1] (< 2^32 each)
    u32 prev_hi = shfl_up_u32((u32)(c >> 32), 1);
    if (lane_id() == 0) prev_hi = spill;
    const u64 v = (u64)(u32)c + prev_hi;
    const u32 limb = w_resolve(v, carry);
    if (p < ns) tot[p] = limb;
    spill = shfl_u32((u32)(c >> 32), WAVE - 1);
  }
}

// ---------------------------------------------------------------------------
hipError_t launch_adj_y(const int* yhdr, const u32* ymant, int NWM, const Dims& dm, const i32* s, u32* Y, u32* Yc,
                        u32* ysq, DevStatus* st, hipStream_t stream) {
  const int threads = 256;
  const size_t lds = (size_t)(threads / WAVE) * (2 * NWM + 2 * dm.nl + 16) * 4;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_adj_y, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adj_y, dim3(1), dim3(threads), lds, stream, yhdr, ymant, NWM, dm, s, Y, Yc, ysq, st);
  return hipGetLastError();
}

hipError_t launch_adj_g(const u32* X, const u32* Yc, const u32* omega, int ostride, const Dims& dm, long eG, u32* ACC,
                        DevStatus* st, hipStream_t stream) {
  const int nl = dm.nl;
  const int nt = 2 * nl + 2, np = nt + nl + 2;
  const size_t lds = (size_t)(nt + 2 * nl + nl + 2 + np + np + 2 + dm.nw) * 4;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_adj_g, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adj_g, dim3(dm.N), dim3(64), lds, stream, X, Yc, omega, ostride, dm, eG, ACC, st);
  return hipGetLastError();
}

hipError_t launch_adj_row(const u32* ACC, const Dims& dm, int i, const i32* h, u32* Z, DevStatus* st,
                          hipStream_t stream) {
  const size_t lds = (size_t)(dm.nw + 2 + dm.nl + 2 + adj_rip_words(dm.nw)) * 4;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_adj_row, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adj_row, dim3(1), dim3(ADJ_ROW_THREADS), lds, stream, ACC, dm, i, h, Z, st);
  return hipGetLastError();
}

hipError_t launch_adj_wprime(const u32* dmu, const i64* dexp, int w, const Dims& dm, const i32* s, i64* wprime,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_adj_wprime, dim3(1), dim3(256), 0, stream, dmu, dexp, w, dm, s, wprime);
  return hipGetLastError();
}

hipError_t launch_adj_da(const u32* dmu, const i64* dexp, const int* dneg, int w, const Dims& dm, const i32* s,
                         const i64* wprime, int j0, int npan, u32* DA, int lda, DevStatus* st, hipStream_t stream) {
  if (npan <= 0) return hipSuccess;
  if (lda < dm.nw) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_adj_da, dim3(dm.N, npan), dim3(64), 0, stream, dmu, dexp, dneg, w, dm, s, wprime, j0, DA, lda,
                     st);
  return hipGetLastError();
}

hipError_t launch_adj_finish(const u32* R, int nr, const u32* Z, const Dims& dm, u32* part, unsigned long long* col,
                             u32* tot, DevStatus* st, hipStream_t stream) {
  const size_t lds = (size_t)(nr + dm.nl) * 4;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_adj_part, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adj_part, dim3(dm.N), dim3(64), lds, stream, R, nr, Z, dm, part, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int ns = 4 * dm.nl + 4;
  hipLaunchKernelGGL(k_adj_colsum, dim3((ns + 255) / 256), dim3(256), 0, stream, part, dm.N, ns, col);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adj_resolve, dim3(1), dim3(64), 0, stream, col, ns, tot);
  return hipGetLastError();
}

hipError_t launch_adj_contract(const u32* dmu, const i64* dexp, const int* dneg, int w, const Dims& dm, const i32* s,
                               i64* wprime, const u32* Z, u32* part, unsigned long long* col, u32* tot,
                               DevStatus* st, hipStream_t stream) {
  hipLaunchKernelGGL(k_adj_wprime, dim3(1), dim3(256), 0, stream, dmu, dexp, w, dm, s, wprime);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nl = dm.nl;
  const size_t per = (size_t)dm.nw + 4 + nl + 2 + 3 * nl + 4;
  int nwv = ADJ_WAVES;
  while (nwv > 1 && nwv * per * 4 > 160 * 1024) --nwv;
  const size_t lds = nwv * per * 4;
  if (lds > 65536) {
    e = hipFuncSetAttribute((const void*)k_adj_contract, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adj_contract, dim3(dm.N), dim3(nwv * 64), lds, stream, dmu, dexp, dneg, w, dm, s, wprime,
                     Z, part, st);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int ns = 4 * nl + 4;
  hipLaunchKernelGGL(k_adj_colsum, dim3((ns + 255) / 256), dim3(256), 0, stream, part, dm.N, ns, col);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adj_resolve, dim3(1), dim3(64), 0, stream, col, ns, tot);
  return hipGetLastError();
}

}  // namespace hl
