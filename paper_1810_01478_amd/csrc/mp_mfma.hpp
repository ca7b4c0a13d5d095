// Exact product of two non-negative multi-limb numbers by one workgroup with
// int8 MFMA (v_mfma_i32_32x32x32_i8), for the products on a single pivot's
// critical path (the reciprocal's Newton steps and remainder).
//
// Each factor x of n limbs is recoded into 4 (n + 1) balanced base-256 digits
// (an (n + 1)-limb two's complement with a zero top limb, so the top digit is
// the final carry), padded with zero digits to whole 32-digit chunks.  With a
// chunks J of a and b chunks c, output block J + c receives the 32 x 32 digit
// convolution of the two chunks.  One MFMA takes, for one a chunk J, the
// Toeplitz matrix A[m][k] = a_(32 J + t(m) - k) and 32 consecutive b chunks
// B[k][n] = b_(32 c_n + k), c_n = O + n - J, so that column n accumulates output
// block O + n for every J (the window of J spans a digits 32 J - 31 .. 32 J + 31,
// so J runs from 0 to the chunk count): a wave owns the 32 blocks O .. O + 31
// (1024 output digits) and steps J over the windows that reach them.  The output digit t(m)
// of MFMA row m is permuted so that lane l, register v holds digit 16 (l >> 5) + v
// of its block: each lane folds 16 digit sums into a 128-bit chunk value plus a
// signed carry, and one wave adds the shifted carries at the end.
#pragma once
#include "mp.hpp"

namespace hl {

typedef int wm_v4i __attribute__((ext_vector_type(4)));
typedef int wm_v16i __attribute__((ext_vector_type(16)));

constexpr int WM_PAD = 64;  // zero bytes on each side of a's reversed digit string

__host__ __device__ __forceinline__ int wm_chunks(int n) { return (4 * (n + 1) + 31) / 32; }
// output blocks 0 .. nJa + nJb - 1 (window nJa with b chunk nJb - 1 reaches the last)
__host__ __device__ __forceinline__ int wm_sets(int na, int nb) { return (wm_chunks(na) + wm_chunks(nb) + 31) / 32; }
// scratch bytes (16-byte aligned pieces): reversed a digits, forward b digits,
// chunk limbs, chunk carries
__host__ __device__ __forceinline__ size_t wm_scratch_bytes(int na, int nb) {
  const size_t ar = (size_t)2 * WM_PAD + 32 * wm_chunks(na);
  const size_t bf = (size_t)32 * wm_chunks(nb);
  const size_t nc = (size_t)64 * wm_sets(na, nb);
  return ar + bf + nc * 16 + nc * 8;
}

// balanced digits 4q .. 4q+3 of the non-negative x (n limbs; limb n reads as 0),
// digit 4q in the low byte; the top digit 4n+3 keeps the sign (it is 0 or 1)
__device__ __forceinline__ u32 wm_digits4(const u32* x, int n, int q) {
  int cin = 0;
  for (int j = 4 * q - 1; j >= 0; --j) {
    const u32 byte = (x[j >> 2] >> (8 * (j & 3))) & 0xffu;
    if (byte != 0x7fu) {
      cin = byte >= 0x80u ? 1 : 0;
      break;
    }
  }
  const u32 limb = q < n ? x[q] : 0u;
  u32 out = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    int v = (int)((limb >> (8 * b)) & 0xffu) + cin;
    if (q < n) {
      cin = v >= 128 ? 1 : 0;
      if (cin) v -= 256;
    } else {
      cin = 0;  // the zero top limb: at most one carry digit, then zeros
    }
    out |= (u32)(v & 0xff) << (8 * b);
  }
  return out;
}

__device__ __forceinline__ wm_v4i wm_window(wm_v4i lo, wm_v4i hi, int aw, int ab) {
  const bool s2 = (aw & 2) != 0, s1 = (aw & 1) != 0;
  const u32 f0 = s2 ? (u32)lo.z : (u32)lo.x, f1 = s2 ? (u32)lo.w : (u32)lo.y;
  const u32 f2 = s2 ? (u32)hi.x : (u32)lo.z, f3 = s2 ? (u32)hi.y : (u32)lo.w;
  const u32 f4 = s2 ? (u32)hi.z : (u32)hi.x, f5 = s2 ? (u32)hi.w : (u32)hi.y;
  const u32 e0 = s1 ? f1 : f0, e1 = s1 ? f2 : f1, e2 = s1 ? f3 : f2, e3 = s1 ? f4 : f3, e4 = s1 ? f5 : f4;
  wm_v4i o;
  o.x = (int)__builtin_amdgcn_alignbyte(e1, e0, (u32)ab);
  o.y = (int)__builtin_amdgcn_alignbyte(e2, e1, (u32)ab);
  o.z = (int)__builtin_amdgcn_alignbyte(e3, e2, (u32)ab);
  o.w = (int)__builtin_amdgcn_alignbyte(e4, e3, (u32)ab);
  return o;
}

// out[0..nout) = a b mod 2^(32 nout); a, b, out and scratch in LDS (out may not
// alias a or b); every thread of the workgroup calls it; ends with a barrier.
// Only the output sets (256 limbs each) below nout are formed.  lo_limb > 0:
// the sets below the one holding limb lo_limb are left out too, and limbs lo ..
// nout - 1 (lo = lo_limb rounded down to a set) receive the product's limbs
// without the carry out of the part below lo (a 16-digit chunk's value is below
// 2^151 in magnitude, so the result differs from (a b) >> 32 lo, modulo
// 2^(32 (nout - lo)), by less than 2^24 units of limb lo); out[0..lo) is not
// written.
__device__ __forceinline__ void wg_mfma_mul(const u32* a, int na, const u32* b, int nb, u32* out, int nout, u32* scratch,
                                            int lo_limb = 0) {
  const int nth = blockDim.x, tid = threadIdx.x;
  const int nwv = nth / WAVE, w = wave_id(), l = lane_id(), h = l >> 5, n = l & 31;
  const int nJa = wm_chunks(na), nJb = wm_chunks(nb), nsets = wm_sets(na, nb);
  const int set0 = lo_limb > 0 ? lo_limb / 256 : 0;
  const int set1 = (nout + 255) / 256 < nsets ? (nout + 255) / 256 : nsets;
  const int lo = 256 * set0;
  const int SA = 32 * nJa;
  int8_t* ar = (int8_t*)scratch;                 // WM_PAD + SA + WM_PAD
  int8_t* bf = ar + 2 * WM_PAD + SA;             // 32 nJb
  u32* olo = (u32*)(bf + 32 * nJb);              // 64 nsets chunks x 4 limbs
  i64* ocw = (i64*)(olo + 256 * nsets);          // 64 nsets carries
  // digits: a reversed (byte WM_PAD + y is digit SA-1-y), b forward
  {
    u32* ar4 = (u32*)ar;
    const int nw4 = (2 * WM_PAD + SA) / 4;
    for (int g = tid; g < nw4; g += nth) {
      const int y = 4 * g - WM_PAD;  // bytes y .. y+3: digits SA-1-y .. SA-4-y, limb SA/4-1-y/4
      u32 v = 0;
      if (y >= 0 && y < SA) {
        const int q = SA / 4 - 1 - y / 4;
        v = q <= na ? __builtin_bswap32(wm_digits4(a, na, q)) : 0u;
      }
      ar4[g] = v;
    }
    u32* bf4 = (u32*)bf;
    for (int g = tid; g < 8 * nJb; g += nth) bf4[g] = g <= nb ? wm_digits4(b, nb, g) : 0u;
  }
  __syncthreads();
  // the MFMA row of this lane's Toeplitz operand and its output digit
  const int tm = 16 * ((n >> 2) & 1) + 4 * (n >> 3) + (n & 3);
  // a digits 32 J + tm - 16 h - x, x = 0..15, are the reversed bytes y0 .. y0 + 15
  // with y0 = yb - 32 J: the 16-byte alignment offset is the same for every J
  const int yb = WM_PAD + SA - 1 - tm + 16 * h;
  const int abase = yb & ~15, aw = (yb & 15) >> 2, ab = yb & 3;
  const wm_v4i zero4 = (wm_v4i){0, 0, 0, 0};
  for (int set = set0 + w; set < set1; set += nwv) {
    const int O = 32 * set;
    // window J holds a digits 32 J - 31 .. 32 J + 31, so J runs to nJa
    int J0 = O - nJb + 1;
    if (J0 < 0) J0 = 0;
    int J1 = O + 31;
    if (J1 > nJa) J1 = nJa;
    // raw operands of window J: the two 16-byte pieces of a's reversed digits
    // and b's chunk (zero outside b).  Beyond J1 they are never used, so the a
    // pieces are read at J1 and only the b predicate keeps its true index.
    auto load = [&](int J, wm_v4i& lo, wm_v4i& hi, wm_v4i& bv) {
      const int Ja = J <= J1 ? J : J1;
      lo = *(const wm_v4i*)(ar + abase - 32 * Ja);
      hi = *(const wm_v4i*)(ar + abase - 32 * Ja + 16);
      const int c = O + n - J;
      bv = zero4;
      if (c >= 0 && c < nJb) bv = *(const wm_v4i*)(bf + 32 * c + 16 * h);
    };
    // two windows per half-step into two accumulators; two register sets (A, B)
    // take turns, so the next pair's operands load while this pair's MFMAs
    // issue.  acc0 + acc1 is the same exact sum as one accumulator.
    wm_v16i acc0 = (wm_v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    wm_v16i acc1 = acc0;
    wm_v4i la0, ha0, ba0, la1, ha1, ba1;  // set A: windows J, J + 1
    wm_v4i lb0, hb0, bb0, lb1, hb1, bb1;  // set B: windows J + 2, J + 3
    load(J0, la0, ha0, ba0);
    load(J0 + 1, la1, ha1, ba1);
    for (int J = J0; J <= J1; J += 4) {
      load(J + 2, lb0, hb0, bb0);
      load(J + 3, lb1, hb1, bb1);
      acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(wm_window(la0, ha0, aw, ab), ba0, acc0, 0, 0, 0);
      if (J + 1 <= J1)
        acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(wm_window(la1, ha1, aw, ab), ba1, acc1, 0, 0, 0);
      if (J + 2 > J1) break;
      load(J + 4, la0, ha0, ba0);
      load(J + 5, la1, ha1, ba1);
      acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(wm_window(lb0, hb0, aw, ab), bb0, acc0, 0, 0, 0);
      if (J + 3 <= J1)
        acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(wm_window(lb1, hb1, aw, ab), bb1, acc1, 0, 0, 0);
    }
    const wm_v16i acc = acc0 + acc1;
    // lane: output block O + n, digits 16 h .. 16 h + 15 = chunk 2 (O + n) + h
    i64 dd[4] = {0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 16; ++v) dd[v >> 2] += (i64)acc[v] << (8 * (v & 3));
    const __int128 X = (__int128)dd[0] + ((__int128)dd[1] << 32);
    const __int128 Y = (__int128)dd[2] + ((__int128)dd[3] << 32) + (__int128)(i64)(X >> 64);
    const u64 lo = (u64)X, hi = (u64)Y;
    const int ch = 2 * (O + n) + h;
    *(uint4*)(olo + 4 * ch) = make_uint4((u32)lo, (u32)(lo >> 32), (u32)hi, (u32)(hi >> 32));
    ocw[ch] = (i64)(Y >> 64);
  }
  __syncthreads();
  // out = sum_ch (olo_ch + ocw_ch 2^128) 2^(128 ch): the chunk limbs plus the
  // positive carries plus the complement of the negative ones, plus one at the
  // lowest limb formed (chunks 64 set0 .. 64 set1 - 1; limb q of the result is
  // value(q - lo))
  const int ch0 = 64 * set0, ch1 = 64 * set1;
  auto value = [=](int q) -> u64 {
    const int p = q + lo;
    u64 v = p < 4 * ch1 ? olo[p] : 0u;
    u32 pos = 0, neg = 0;
    const int c = (p >> 2) - 1, j = p & 3;
    if (c >= ch0 && c < ch1 && j < 2) {
      const i64 cw = ocw[c];
      const u64 m = cw < 0 ? (u64)(-cw) : (u64)cw;
      const u32 word = (u32)(m >> (32 * j));
      if (cw < 0) neg = word; else pos = word;
    }
    v += (u64)pos + (u64)(~neg);
    if (q == 0) v += 1;
    return v;
  };
  const int nres = nout - lo;
  u32* const outl = out + lo;
  // resolved by the whole workgroup, the digit strings (no longer needed) holding
  // the ripple table; one wave if they are too short for it
  if ((size_t)8 * ((nres + WAVE - 1) / WAVE) <= (size_t)2 * WM_PAD + 32 * (nJa + nJb)) {
    wg_resolve(nres, value, outl, (u32*)ar);
    return;
  }
  if (w == 0) {
    u32 carry = 0;
    u64 vn = value(l);
    for (int base = 0; base < nres; base += WAVE) {
      const int p = base + l;
      const u64 v = vn;
      vn = p + WAVE < nres ? value(p + WAVE) : 0ull;
      const u32 limb = w_resolve(v, carry);
      if (p < nres) outl[p] = limb;
    }
  }
  __syncthreads();
}

}  // namespace hl
