// Multi-limb integer primitives for gfx950, at wave (64-lane) level.
//
// Numbers are little-endian arrays of uint32 limbs.  Signed quantities are two's
// complement over a fixed limb count.  Every routine here is exact integer
// arithmetic; the rounding points of the method live in the kernels that call
// them, never in here.
//
// Column sums: a product a*b is formed by product scanning.  Output column t is
// sum_x a[x] b[t-x], accumulated as a 96-bit value (64-bit low word with a
// 32-bit count of its carries).  A run of 64 consecutive columns is turned into
// limbs by one wave at a time: the three 32-bit words of column t land on
// positions t, t+1, t+2; the per-position sums are split into a limb and a carry
// word; the carry words move up one lane; the single-bit carries that remain are
// resolved across the 64 lanes with two ballots and one 64-bit add
// (carry-lookahead: with G = generate and P = propagate masks, the carries into
// the lanes are ((G|P) + G) ^ (G|P) ^ G).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hl {

typedef uint32_t u32;
typedef uint64_t u64;
typedef int64_t i64;
typedef int32_t i32;

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / WAVE; }

__device__ __forceinline__ u64 ballot64(bool p) { return __ballot(p); }

// make this wave's global and LDS writes visible to its other lanes
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// 96-bit accumulate: (lo, hi) += a * b.  v_mad_u64_u32 writes its carry out to
// VCC, which v_addc_co_u32 folds into the carry count.
__device__ __forceinline__ void mac96(u64& lo, u32& hi, u32 a, u32 b) {
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t"
      "v_addc_co_u32 %1, vcc, 0, %1, vcc"
      : "+v"(lo), "+v"(hi)
      : "v"(a), "v"(b)
      : "vcc");
}

// Column sum sum_{x=x0..x1} a[x] b[t-x] into (lo, hi), unrolled by four.
__device__ __forceinline__ void col_sum(const u32* a, const u32* b, int t, int x0, int x1, u64& lo,
                                        u32& hi) {
  int x = x0;
  for (; x + 3 <= x1; x += 4) {
    const u32 a0 = a[x], a1 = a[x + 1], a2 = a[x + 2], a3 = a[x + 3];
    const u32* bb = b + (t - x);
    const u32 b0 = bb[0], b1 = bb[-1], b2 = bb[-2], b3 = bb[-3];
    mac96(lo, hi, a0, b0);
    mac96(lo, hi, a1, b1);
    mac96(lo, hi, a2, b2);
    mac96(lo, hi, a3, b3);
  }
  for (; x <= x1; ++x) mac96(lo, hi, a[x], b[t - x]);
}

__device__ __forceinline__ u32 shfl_up_u32(u32 v, int d) { return (u32)__shfl_up((int)v, d, WAVE); }
__device__ __forceinline__ u32 shfl_u32(u32 v, int src) { return (u32)__shfl((int)v, src, WAVE); }
__device__ __forceinline__ u32 shfl_down_u32(u32 v, int d) { return (u32)__shfl_down((int)v, d, WAVE); }

__device__ __forceinline__ int wave_max_i32(int v) {
  for (int o = 32; o > 0; o >>= 1) {
    int w = __shfl_xor(v, o, WAVE);
    v = w > v ? w : v;
  }
  return v;
}
__device__ __forceinline__ int wave_min_i32(int v) {
  for (int o = 32; o > 0; o >>= 1) {
    int w = __shfl_xor(v, o, WAVE);
    v = w < v ? w : v;
  }
  return v;
}
__device__ __forceinline__ int wave_or_i32(int v) {
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, WAVE);
  return v;
}

// ---------------------------------------------------------------------------
// Carry resolution of one 64-position chunk.
//   v     : this lane's position value, v < 2^63
//   carry : in  = wave-uniform value added at position 0 of the chunk (< 2^32)
//           out = wave-uniform carry into position 64 (< 2^31 + 1)
// returns this lane's limb.
__device__ __forceinline__ u32 w_resolve(u64 v, u32& carry) {
  const int l = lane_id();
  const u32 limb0 = (u32)v;
  const u32 c1 = (u32)(v >> 32);
  u32 cprev = shfl_up_u32(c1, 1);
  if (l == 0) cprev = carry;
  const u64 s2 = (u64)limb0 + cprev;
  const u32 limb1 = (u32)s2;
  const bool g = (s2 >> 32) != 0;
  const u64 G = ballot64(g);
  const u64 Pm = ballot64(limb1 == 0xffffffffu);
  const u64 A = G | Pm;
  const u64 S = A + G;
  const u64 cin = S ^ A ^ G;
  const u32 cout = (S < A) ? 1u : 0u;
  carry = shfl_u32(c1, WAVE - 1) + cout;
  return limb1 + (u32)((cin >> l) & 1ull);
}

// ---------------------------------------------------------------------------
// Streaming product of two unsigned numbers a (na limbs) and b (nb limbs), both
// readable by every lane (LDS or global).  Column chunks ch = 0..nch-1 (64
// columns each) are formed in order; sink(ch, limb) receives this lane's limb.
// pre(ch, lo, hi) may add non-negative terms to a column before resolution.
// The result is (a*b + added terms) mod 2^(32*64*nch).
struct NoPre {
  __device__ __forceinline__ void operator()(int, u64&, u32&) const {}
};

template <class Sink, class Pre = NoPre>
__device__ void w_mul_stream(const u32* a, int na, const u32* b, int nb, int nch, Sink sink,
                             Pre pre = Pre()) {
  const int l = lane_id();
  u32 carry = 0;
  u32 sp_mid = 0, sp_hi62 = 0, sp_hi63 = 0;  // spills from the previous chunk
  for (int ch = 0; ch < nch; ++ch) {
    const int t = ch * WAVE + l;
    u64 lo = 0;
    u32 hi = 0;
    if (na > 0 && nb > 0 && t < na + nb - 1) {
      int x0 = t - (nb - 1);
      if (x0 < 0) x0 = 0;
      const int x1 = t < na - 1 ? t : na - 1;
      col_sum(a, b, t, x0, x1, lo, hi);
    }
    pre(ch, lo, hi);
    const u32 w0 = (u32)lo, w1 = (u32)(lo >> 32), w2 = hi;
    u32 m1 = shfl_up_u32(w1, 1);   // word 1 of column t-1
    u32 h2 = shfl_up_u32(w2, 2);   // word 2 of column t-2
    if (l == 0) { m1 = sp_mid; h2 = sp_hi62; }
    if (l == 1) { h2 = sp_hi63; }
    const u64 v = (u64)w0 + m1 + h2;
    const u32 limb = w_resolve(v, carry);
    sink(ch, limb);
    sp_mid = shfl_u32(w1, WAVE - 1);
    sp_hi62 = shfl_u32(w2, WAVE - 2);
    sp_hi63 = shfl_u32(w2, WAVE - 1);
  }
}

// Full product into out[0 .. nout) (nout <= 64*ceil(nout/64) is written up to nout).
__device__ __forceinline__ void w_mul(const u32* a, int na, const u32* b, int nb, u32* out, int nout) {
  const int nch = (nout + WAVE - 1) / WAVE;
  w_mul_stream(a, na, b, nb, nch, [&](int ch, u32 limb) {
    const int p = ch * WAVE + lane_id();
    if (p < nout) out[p] = limb;
  });
}

// ---------------------------------------------------------------------------
// Element-wise helpers.  All lanes of the wave call them; out may alias in only
// where stated.

__device__ __forceinline__ void w_copy(const u32* src, u32* dst, int n) {
  for (int p = lane_id(); p < n; p += WAVE) dst[p] = src[p];
}
__device__ __forceinline__ void w_fill(u32* dst, int n, u32 v) {
  for (int p = lane_id(); p < n; p += WAVE) dst[p] = v;
}

// out = a + b + cin (mod 2^(32n)); a, b zero-extended from na, nb; out may alias a or b.
// returns the carry out of the top limb.
__device__ __forceinline__ u32 w_add(const u32* a, int na, const u32* b, int nb, u32* out, int n,
                                     u32 cin = 0) {
  u32 carry = cin;
  for (int base = 0; base < n; base += WAVE) {
    const int p = base + lane_id();
    u64 v = 0;
    if (p < n) {
      if (p < na) v += a[p];
      if (p < nb) v += b[p];
    }
    const u32 limb = w_resolve(v, carry);
    if (p < n) out[p] = limb;
  }
  return carry;
}

// out = a - b (mod 2^(32n)), a and b two's complement over n limbs (b sign
// extended from nb with sign bit sb); out may alias.
__device__ __forceinline__ void w_sub(const u32* a, const u32* b, u32* out, int n) {
  u32 carry = 1;
  for (int base = 0; base < n; base += WAVE) {
    const int p = base + lane_id();
    u64 v = 0;
    if (p < n) v = (u64)a[p] + (u64)(~b[p]);
    const u32 limb = w_resolve(v, carry);
    if (p < n) out[p] = limb;
  }
}

// x = -x (mod 2^(32n)), in place.
__device__ __forceinline__ void w_neg(u32* x, int n) {
  u32 carry = 1;
  for (int base = 0; base < n; base += WAVE) {
    const int p = base + lane_id();
    u64 v = (p < n) ? (u64)(~x[p]) : 0;
    const u32 limb = w_resolve(v, carry);
    if (p < n) x[p] = limb;
  }
}

// x += v * 2^(32*pos) (mod 2^(32n)), v < 2^32, in place.
__device__ __forceinline__ void w_add_word(u32* x, int n, int pos, u32 v) {
  u32 carry = 0;
  for (int base = (pos / WAVE) * WAVE; base < n; base += WAVE) {
    const int p = base + lane_id();
    u64 s = (p < n) ? (u64)x[p] : 0;
    if (p == pos) s += v;
    const u32 limb = w_resolve(s, carry);
    if (p < n) x[p] = limb;
    if (carry == 0 && base + WAVE > pos) break;
  }
}

// ---------------------------------------------------------------------------
// Carry resolution by a whole workgroup.  out[p] = limb p of
// sum_{p < n} v(p) 2^(32 p) mod 2^(32 n), every v(p) < 2^64.  Limb p receives
// the low word of v(p), the high word of v(p - 1) and a one-bit ripple from
// below; only the ripple crosses a 64-limb chunk, so the chunks are spread over
// the waves: pass 1 records each chunk's carry-out for a ripple-in of 0 and of 1
// and the high word entering it, pass 2 (wave 0) chains the ripples with one
// ballot per 64 chunks, pass 3 writes the limbs.  v(p) may read out[p] (each
// chunk reads its own limbs before writing them) but no other limb of out.
// rip: 2 ceil(n / 64) words of LDS.  All threads call it; it ends with a barrier.
template <class V>
__device__ __forceinline__ void wg_resolve(int n, V value, u32* out, u32* rip) {
  const int l = lane_id(), w = wave_id(), nwv = blockDim.x / WAVE;
  const int nq = (n + WAVE - 1) / WAVE;
  // the generate and propagate masks of chunk k (ripple in excluded)
  auto masks = [&](int k, u32 hin, u64& A, u64& G, u64& s2) {
    const int p = WAVE * k + l;
    const u64 v = p < n ? value(p) : 0ull;
    u32 cprev = shfl_up_u32((u32)(v >> 32), 1);
    if (l == 0) cprev = hin;
    s2 = (u64)(u32)v + cprev;
    G = ballot64((s2 >> 32) != 0);
    A = G | ballot64((u32)s2 == 0xffffffffu);
  };
  for (int k = w; k < nq; k += nwv) {
    u32 hin = 0;
    if (l == 0 && k > 0) hin = (u32)(value(WAVE * k - 1) >> 32);
    hin = shfl_u32(hin, 0);
    u64 A, G, s2;
    masks(k, hin, A, G, s2);
    const u64 S1 = A + G;
    const u32 g = S1 < A ? 1u : 0u;                  // carry out with ripple 0
    const u32 t = (g || S1 == ~0ull) ? 1u : 0u;      // with ripple 1
    if (l == 0) {
      rip[2 * k] = g | (t << 1);
      rip[2 * k + 1] = hin;
    }
  }
  __syncthreads();
  if (w == 0) {
    u32 cg = 0;
    for (int base = 0; base < nq; base += WAVE) {
      const int k = base + l;
      const u32 f = k < nq ? rip[2 * k] : 0u;
      const u64 G2 = ballot64(f & 1u), A2 = ballot64((f >> 1) & 1u);
      const u64 S1 = A2 + G2, S = S1 + cg;
      const u64 cv = S ^ A2 ^ G2;   // ripple into each chunk
      if (k < nq) rip[2 * k] = f | ((u32)((cv >> l) & 1ull) << 2);
      cg = (S1 < A2 || (cg && S == 0)) ? 1u : 0u;
    }
  }
  __syncthreads();
  for (int k = w; k < nq; k += nwv) {
    const u32 c = (rip[2 * k] >> 2) & 1u;
    u64 A, G, s2;
    masks(k, rip[2 * k + 1], A, G, s2);
    const u64 cin = (A + G + c) ^ A ^ G;
    const int p = WAVE * k + l;
    if (p < n) out[p] = (u32)s2 + (u32)((cin >> l) & 1ull);
  }
  __syncthreads();
}

// workgroup forms of the carry loops above (same results); rip as for wg_resolve
__device__ __forceinline__ void wg_add(const u32* a, int na, const u32* b, int nb, u32* out, int n, u32* rip) {
  wg_resolve(n, [=](int p) -> u64 { return (u64)(p < na ? a[p] : 0u) + (u64)(p < nb ? b[p] : 0u); }, out, rip);
}
__device__ __forceinline__ void wg_sub(const u32* a, const u32* b, u32* out, int n, u32* rip) {
  wg_resolve(n, [=](int p) -> u64 { return (u64)a[p] + (u64)(~b[p]) + (p == 0 ? 1u : 0u); }, out, rip);
}
__device__ __forceinline__ void wg_neg(u32* x, int n, u32* rip) {
  wg_resolve(n, [=](int p) -> u64 { return (u64)(~x[p]) + (p == 0 ? 1u : 0u); }, x, rip);
}

// Limb j of (x >> s) for x of nx limbs (logical shift, zero fill), s >= 0.
__device__ __forceinline__ u32 limb_shr(const u32* x, int nx, long s, int j) {
  const long q = s >> 5;
  const int r = (int)(s & 31);
  const long i0 = j + q;
  u32 lo = (i0 >= 0 && i0 < nx) ? x[i0] : 0u;
  if (r == 0) return lo;
  u32 hi = (i0 + 1 >= 0 && i0 + 1 < nx) ? x[i0 + 1] : 0u;
  return (lo >> r) | (hi << (32 - r));
}
// Limb j of (x << s) for x of nx limbs, s >= 0.
__device__ __forceinline__ u32 limb_shl(const u32* x, int nx, long s, int j) {
  const long q = s >> 5;
  const int r = (int)(s & 31);
  const long i0 = (long)j - q;
  u32 hi = (i0 >= 0 && i0 < nx) ? x[i0] : 0u;
  if (r == 0) return hi;
  u32 lo = (i0 - 1 >= 0 && i0 - 1 < nx) ? x[i0 - 1] : 0u;
  return (hi << r) | (lo >> (32 - r));
}

// dst[0..nd) = src >> s (s may be negative: left shift).  dst must not alias src.
__device__ __forceinline__ void w_shift_right(const u32* src, int ns, long s, u32* dst, int nd) {
  for (int j = lane_id(); j < nd; j += WAVE)
    dst[j] = s >= 0 ? limb_shr(src, ns, s, j) : limb_shl(src, ns, -s, j);
}
// the same by every thread of the workgroup; ends with a barrier
__device__ __forceinline__ void wg_shift_right(const u32* src, int ns, long s, u32* dst, int nd) {
  for (int j = threadIdx.x; j < nd; j += blockDim.x)
    dst[j] = s >= 0 ? limb_shr(src, ns, s, j) : limb_shl(src, ns, -s, j);
  __syncthreads();
}

// number of significant bits of x (0 for x == 0)
__device__ __forceinline__ int w_bitlen(const u32* x, int n) {
  int top = -1;
  for (int p = lane_id(); p < n; p += WAVE)
    if (x[p]) top = p;
  top = wave_max_i32(top);
  if (top < 0) return 0;
  return top * 32 + (32 - __clz((int)x[top]));
}

__device__ __forceinline__ bool w_is_zero(const u32* x, int n) {
  int nz = 0;
  for (int p = lane_id(); p < n; p += WAVE) nz |= (x[p] != 0);
  return wave_or_i32(nz) == 0;
}

// sign of (a - b) for unsigned a, b of n limbs: -1, 0, 1
__device__ __forceinline__ int w_cmp(const u32* a, const u32* b, int n) {
  int top = -1;
  for (int p = lane_id(); p < n; p += WAVE)
    if (a[p] != b[p]) top = p;
  top = wave_max_i32(top);
  if (top < 0) return 0;
  return a[top] > b[top] ? 1 : -1;
}

// bit s of x (0 beyond the array)
__device__ __forceinline__ u32 get_bit(const u32* x, int n, long s) {
  const long q = s >> 5;
  if (s < 0 || q >= n) return 0;
  return (x[q] >> (s & 31)) & 1u;
}

// ---------------------------------------------------------------------------
// Workgroup-level product: the waves of the block form the column sums of
// interleaved 64-column chunks into LDS (3 words per column), then wave 0
// turns them into limbs.  All threads of the block must call it.
// colbuf: 3 * nout words of LDS.  out may not alias a or b.
__device__ __forceinline__ void g_mul(const u32* a, int na, const u32* b, int nb, u32* out, int nout,
                                      u32* colbuf) {
  const int w = wave_id(), nwv = blockDim.x / WAVE, l = lane_id();
  const int nch = (nout + WAVE - 1) / WAVE;
  for (int ch = w; ch < nch; ch += nwv) {
    const int t = ch * WAVE + l;
    u64 lo = 0;
    u32 hi = 0;
    if (t < na + nb - 1) {
      int x0 = t - (nb - 1);
      if (x0 < 0) x0 = 0;
      const int x1 = t < na - 1 ? t : na - 1;
      col_sum(a, b, t, x0, x1, lo, hi);
    }
    if (t < nout) {
      colbuf[3 * t] = (u32)lo;
      colbuf[3 * t + 1] = (u32)(lo >> 32);
      colbuf[3 * t + 2] = hi;
    }
  }
  __syncthreads();
  if (w == 0) {
    u32 carry = 0;
    for (int ch = 0; ch < nch; ++ch) {
      const int p = ch * WAVE + l;
      u64 v = 0;
      if (p < nout) {
        v = colbuf[3 * p];
        if (p >= 1) v += colbuf[3 * (p - 1) + 1];
        if (p >= 2) v += colbuf[3 * (p - 2) + 2];
      }
      const u32 limb = w_resolve(v, carry);
      if (p < nout) out[p] = limb;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Balanced digits 4q .. 4q+3 of the nl-limb two's complement x, packed in a
// word (digit 4q in the low byte).  Digit j is byte_j + c_j - 256 c_{j+1} with
// c_{j+1} = [byte_j + c_j >= 128], except the top digit, which keeps the sign.
// The carry into digit 4q is found by looking down past bytes 0x7f.
__device__ __forceinline__ u32 balanced_digits4(const u32* __restrict__ x, int nl, int q) {
  int cin = 0;
  for (int j = 4 * q - 1; j >= 0; --j) {
    const u32 byte = (x[j >> 2] >> (8 * (j & 3))) & 0xffu;
    if (byte != 0x7fu) {
      cin = byte >= 0x80u ? 1 : 0;
      break;
    }
  }
  const u32 limb = x[q];
  const int top = 4 * nl - 1;
  u32 out = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int j = 4 * q + b;
    int v;
    if (j == top) {
      v = (int)(int8_t)(limb >> 24) + cin;
      cin = 0;
    } else {
      v = (int)((limb >> (8 * b)) & 0xffu) + cin;
      cin = v >= 128 ? 1 : 0;
      if (cin) v -= 256;
    }
    out |= (u32)(v & 0xff) << (8 * b);
  }
  return out;
}

}  // namespace hl
