// Karatsuba form of the exact Schur update (see KaraArgs): the digit panels of
// the split factors, the recombination of the stored products into the
// trailing matrix, and the launcher around the digit-sum GEMMs (k_upd_kara, in
// k_upd_mfma.hip).
#include <utility>

#include "hl_kernels.hpp"

namespace hl {

// Digits of the halves: limb q of a factor holds its balanced digits 4q..4q+3;
// those below h = 4 hq go to the lo panel, the others to the hi panel at digit
// 4q - h.  One thread per (limb, row, panel column), as recode_body, for rows
// r0 .. NT - 1 (the GEMMs of a launch read no row below its first tile row).
__global__ void k_recode_kara(const u32* __restrict__ src, size_t lds, int npan, int NT, int nrows, int nl, int pad,
                              int hq, int8_t* __restrict__ lo, int8_t* __restrict__ hi, int r0) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int il = (int)(gid & 15);
  const size_t t = gid >> 4;
  const int nr = NT - r0;
  const int row = r0 + (int)(t % nr), q = (int)(t / nr);
  if (q >= nl) return;
  const size_t rstride = (size_t)NT * 16;
  const int qq = q < hq ? q : q - hq;
  int8_t* d = (q < hq ? lo : hi) + (size_t)(pad + 4 * qq) * rstride + (size_t)row * 16 + il;
  u32 v = 0;
  if (il < npan && row < nrows) v = balanced_digits4(src + (size_t)il * lds + (size_t)row * nl, nl, q);
#pragma unroll
  for (int b = 0; b < 4; ++b) d[(size_t)b * rstride] = (int8_t)(v >> (8 * b));
}

// floor((x + 128) / 256) for -512 <= x + 128: the balanced carry out of a
// digit position holding x
__device__ __forceinline__ int bal_carry(int x) { return (x + 640) / 256 - 2; }

// mid = lo + hi recoded into h + 1 balanced digits: sigma_j = lo_j + hi_j in
// [-256, 254], digit_j = sigma_j + c_j - 256 c_{j+1}, c_{j+1} = bal_carry(sigma_j
// + c_j) in {-1, 0, 1}, c_0 = 0; the top digit h is c_h.  One thread per (group
// of digits 4g..4g+3, row), g = 0..h/4, for the row's 16 panel columns at once
// (16-byte loads and stores of a slice row); the carry into 4g of each column
// is found by looking down to the nearest position whose carry out does not
// depend on the carry in, then carrying up from there.
__device__ __forceinline__ int sig_byte(const uint4& a, const uint4& b, int col) {
  const u32 wa = col < 4 ? a.x : col < 8 ? a.y : col < 12 ? a.z : a.w;
  const u32 wb = col < 4 ? b.x : col < 8 ? b.y : col < 12 ? b.z : b.w;
  const int sh = 8 * (col & 3);
  return (int)(int8_t)(wa >> sh) + (int)(int8_t)(wb >> sh);
}

__device__ __forceinline__ void kara_mid_body(const int8_t* __restrict__ lo, const int8_t* __restrict__ hi, int NT,
                                              int pad, int h, int8_t* __restrict__ mid, int r0) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nr = NT - r0;
  const int row = r0 + (int)(gid % nr), g = (int)(gid / nr);
  if (g > h / 4) return;
  const size_t rs = (size_t)NT * 16, off = (size_t)row * 16;
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  auto ld = [&](const int8_t* P, int j) -> uint4 { return j < h ? *(const uint4*)(P + (size_t)(pad + j) * rs + off) : z; };
  const int j0 = 4 * g;
  int c[16], js[16];
  unsigned open = 0xffffu;  // columns whose look-down has not ended
#pragma unroll
  for (int col = 0; col < 16; ++col) {
    c[col] = 0;
    js[col] = -1;
  }
  int jmin = j0;
  for (int j = j0 - 1; j >= 0 && open; --j) {
    const uint4 a = ld(lo, j), b = ld(hi, j);
#pragma unroll
    for (int col = 0; col < 16; ++col) {
      if (!((open >> col) & 1u)) continue;
      const int sj = sig_byte(a, b, col);
      if (bal_carry(sj - 1) == bal_carry(sj + 1)) {
        c[col] = bal_carry(sj);  // carry into j + 1
        js[col] = j;
        open &= ~(1u << col);
      }
    }
    jmin = j;
  }
  // carry up from each column's js + 1 to j0 (columns left open start at 0 with c = 0)
  for (int j = jmin < j0 ? jmin : j0; j < j0; ++j) {
    const uint4 a = ld(lo, j), b = ld(hi, j);
#pragma unroll
    for (int col = 0; col < 16; ++col)
      if (j > js[col]) c[col] = bal_carry(sig_byte(a, b, col) + c[col]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint4 a = ld(lo, j0 + q), b = ld(hi, j0 + q);
    u32 w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int col = 0; col < 16; ++col) {
      const int x = sig_byte(a, b, col) + c[col];
      const int cn = bal_carry(x);
      w[col >> 2] |= (u32)((x - 256 * cn) & 0xff) << (8 * (col & 3));
      c[col] = cn;
    }
    *(uint4*)(mid + (size_t)(pad + j0 + q) * rs + off) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

__global__ void k_kara_mid(const int8_t* __restrict__ lo, const int8_t* __restrict__ hi, int NT, int pad, int h,
                           int8_t* __restrict__ mid, int r0) {
  kara_mid_body(lo, hi, NT, pad, h, mid, r0);
}

// the mid children of every level-(l-1) panel (blockIdx.y, both sides): lo and
// hi child of n = S/2^(l-1) + extra digits, the hi child n - S/2^l of them
__global__ void k_kara_mid_lv(KaraArgs k, int l, int r0) {
  const int nq = kara_products(l - 1), y = blockIdx.y, side = y / nq, q = y - side * nq;
  const int s = k.m.S >> l;
  int8_t* lo = k.pan[l] + (size_t)(side * 3 * nq + 3 * q) * k.pan_stride[l];
  kara_mid_body(lo, lo + k.pan_stride[l], k.m.NT, k.m.pad, s + kara_extra(q, l - 1), lo + 2 * k.pan_stride[l], r0);
}

// Level l - 1 to level l: every panel q (blockIdx.y, both sides) has
// n = S/2^(l-1) + extra digits; slices [0, s) go to its lo child, [s, n) to its hi
// child (digit j - s), s = S/2^l.  One thread per 16 bytes of a slice row
// r0 .. NT - 1.
__global__ void k_digit_split(KaraArgs k, int l, int r0) {
  const int nq = kara_products(l - 1), y = blockIdx.y, side = y / nq, q = y - side * nq;
  const int s = k.m.S >> l, n = 2 * s + kara_extra(q, l - 1), NT = k.m.NT, pad = k.m.pad;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nr = NT - r0;
  const int j = (int)(gid / nr), row = r0 + (int)(gid % nr);
  if (j >= n) return;
  const size_t rs = (size_t)NT * 16;
  const int8_t* src = k.pan[l - 1] + (size_t)y * k.pan_stride[l - 1];
  int8_t* lo = k.pan[l] + (size_t)(side * 3 * nq + 3 * q) * k.pan_stride[l];
  const uint4 v = *(const uint4*)(src + (size_t)(pad + j) * rs + (size_t)row * 16);
  int8_t* d = j < s ? lo + (size_t)(pad + j) * rs : lo + k.pan_stride[l] + (size_t)(pad + j - s) * rs;
  *(uint4*)(d + (size_t)row * 16) = v;
}

// The combination a -= sum_p c_p(Y) P_p as terms (product p, power of Y, sign
// of the subtraction), sorted by product: c_p = prod_l f_(c_l)(Y^(2^(L-l))) over
// the base-3 digits c_l of p (level 1 most significant), f_lo(z) = 1 - z,
// f_hi(z) = z^2 - z, f_mid(z) = z.  The powers of one product are distinct (a
// level's powers differ by at most 1 in units of the next finer level's 2), so
// c_p has 2^(lo or hi levels) terms, 5^L in all.
struct KaTerm {
  int p, pw, sg;
};
template <int LV>
struct KaPoly {
  static constexpr int NP = kara_products(LV);
  static constexpr int NT = LV == 1 ? 5 : (LV == 2 ? 25 : (LV == 3 ? 125 : 625));
  KaTerm t[NT];
  int first[NP + 1];
  constexpr KaPoly() : t(), first() {
    int n = 0;
    for (int p = 0; p < NP; ++p) {
      first[p] = n;
      int pw[16] = {}, cf[16] = {}, m = 1;
      pw[0] = 0;
      cf[0] = 1;
      int div = NP / 3;
      for (int l = 1; l <= LV; ++l) {
        const int c = (p / div) % 3;
        div = div / 3;
        const int z = 1 << (LV - l);
        int pw2[16] = {}, cf2[16] = {}, m2 = 0;
        for (int a = 0; a < m; ++a) {
          if (c == 0) {
            pw2[m2] = pw[a]; cf2[m2++] = cf[a];
            pw2[m2] = pw[a] + z; cf2[m2++] = -cf[a];
          } else if (c == 1) {
            pw2[m2] = pw[a] + 2 * z; cf2[m2++] = cf[a];
            pw2[m2] = pw[a] + z; cf2[m2++] = -cf[a];
          } else {
            pw2[m2] = pw[a] + z; cf2[m2++] = cf[a];
          }
        }
        for (int a = 0; a < m2; ++a) {
          pw[a] = pw2[a];
          cf[a] = cf2[a];
        }
        m = m2;
      }
      for (int a = 0; a < m; ++a) t[n++] = KaTerm{p, pw[a], -cf[a]};
    }
    first[NP] = n;
  }
};

// the live entry (r, c) of launch tile lt, or false
__device__ __forceinline__ bool kara_entry(const KaraArgs& k, int C_lo, int lt, int e, int* R, int* C) {
  const UpdArgs& g = k.m.g;
  item_tile(g, C_lo, lt, R, C);
  if (*R * 32 >= k.m.NT) return false;
  const int rg = *R * 32 + (e >> 5), cg = *C * 32 + (e & 31);
  return (!g.tri || rg >= cg) && rg >= g.r_lo && rg < g.r_hi && cg >= g.c_lo && cg < g.c_hi;
}

// add the sign-extended value cv at limb li (even) of the entry at w (limbs
// word-addressed by in_tile), the carry or borrow running on up to limb nw
__device__ __forceinline__ void add_at_limb(u32* w, int r, int c, int li, int nw, i64 cv) {
  if (cv == 0 || li >= nw) return;
  u32* p0 = w + in_tile(r, c, li);
  const u64 x0 = ((u64)p0[1] << 32) | p0[0];
  const u64 y0 = x0 + (u64)cv;
  p0[0] = (u32)y0;
  p0[1] = (u32)(y0 >> 32);
  const u64 add = (cv < 0 ? ~0ull : 0ull) + (y0 < x0 ? 1ull : 0ull);  // 0, 1 or ~0
  if (add == 0) return;
  for (li += 2; li < nw; li += 2) {
    u32* q = w + in_tile(r, c, li);
    const u64 x = ((u64)q[1] << 32) | q[0];
    const u64 y = x + add;
    q[0] = (u32)y;
    q[1] = (u32)(y >> 32);
    if (add == 1 ? (y != 0) : (x != 0)) break;
  }
}

// Add the carries out of all but the last range of product blockIdx.y at the
// first limb of the next range, for every live entry (one thread each).  The
// product then holds its exact value modulo 2^(32 nwp); it is far below
// 2^(32 nwp - 1) in magnitude, so its top slab read as a signed 128-bit
// number gives the exact value, and the last range's carry (its sign
// extension) is not needed.
__global__ __launch_bounds__(256) void k_kara_fix(KaraArgs k, RangeTab rt, int C_lo, int ntiles) {
  const int lt = blockIdx.x >> 2, e = (blockIdx.x & 3) * 256 + threadIdx.x, p = blockIdx.y;
  int R, C;
  if (!kara_entry(k, C_lo, lt, e, &R, &C) || has_error(k.m.g.st)) return;
  const int r = e >> 5, c = e & 31;
  u32* Q = k.prod + ((size_t)lt * kara_products(k.levels) + p) * tile_words(k.nwp);
  const long long* cb = k.m.carry + ((size_t)p * ntiles + lt) * rt.n * 1024 + e;
  for (int w = 0; w + 1 < rt.n; ++w) add_at_limb(Q, r, c, MF_LPB * rt.tb[w + 1], k.nwp, cb[(size_t)w * 1024]);
}

// a -= sum_p c_p(Y) P_p for every live entry of the launch, two lanes per
// entry: lane half h (lane & 1) holds limbs 2h, 2h + 1 of every slab.  Y is O
// slabs, the entry 2^(L+1) segments of O slabs, every product 2 O + 1 slabs
// with a signed top slab.  Output slab m O + jj takes, from term (p, pw),
// product slab (m - pw) O + jj: slab jj for m = pw, O + jj for m = pw + 1, and
// the top slab 2 O at jj = 0 for m = pw + 2.  So the lane pair walks jj, holds
// slab jj of every segment in registers, streams the two slabs jj and O + jj of
// every product through once (each lane its 8 bytes), and stores the segments,
// each with its own running carry; at the end the carry out of segment m
// enters at its successor's first slab.
//
// Memory: the launch tile's products are contiguous (tile lt holds its np
// products, tw words apart) and read through one buffer descriptor: a lane
// offset (the entry, the product) in a register, the slab in a scalar.  The
// products go in groups of G; the loads of group g + NB - 1 are issued before
// group g is added in (NB groups of slabs in registers, NB below), into the
// registers group g - 1 has just used.  Before those loads the accumulators
// pass through empty asm statements (they must hold their values after group
// g - 1 there) and then the lane offset through one more,
// so the compiler neither hoists later loads into the accumulators' registers
// nor keeps 3^L product offsets live; the fence emits no instruction.  Slab
// position 0, the only one that reads the products' top slabs, runs as its own
// copy of the loop body, so the others carry no test for it.
template <int LV>
struct KaComb {
  static constexpr int NP = kara_products(LV);
  static constexpr int G = LV <= 2 ? NP : 3;  // products per load group
  static constexpr int NG = (NP + G - 1) / G;
};
// load groups in registers, NB - 1 of them in flight while one is added in: three
// in the four-level main loop, two where more registers would cost occupancy
// (three levels) or spill (slab position 0, which also holds the top slabs)
template <int LV, bool J0>
struct KaNb {
  static constexpr int NB = LV >= 4 && !J0 ? 3 : 2;
};
template <int LV, bool J0>
using KaBuf = uint2[KaNb<LV, J0>::NB][KaComb<LV>::G][3];

__device__ __forceinline__ void ka_apply(i64 (&s)[2], const uint2& v, int sg, bool top_hi) {
  // top_hi: this lane holds limbs 2, 3 of the top slab, whose limb 3 is signed
  const i64 v1 = top_hi ? (i64)(int)v.y : (i64)v.y;
  if (sg > 0) {
    s[0] += v.x; s[1] += v1;
  } else {
    s[0] -= v.x; s[1] -= v1;
  }
}

typedef unsigned v2u __attribute__((ext_vector_type(2)));

// a lane offset beyond every descriptor's size here: raw buffer loads from it
// return zero (range check on the lane offset)
constexpr u32 kBufferOutOfRange = 0x80000000u;

__device__ __forceinline__ uint2 bld8(__amdgpu_buffer_rsrc_t r, u32 voff, int soff) {
  const v2u v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, soff, 0);
  return make_uint2(v.x, v.y);
}

// the partner lane's value (lanes 2i and 2i + 1 swap)
__device__ __forceinline__ int partner32(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false); }

// Group g's slabs: product p = g G + i at lane offset vo + i tw4; lo slab jj,
// hi slab O + jj, the top slab 2 O at jj = 0.
template <int LV, int GI, bool J0>
__device__ __forceinline__ void ka_load(__amdgpu_buffer_rsrc_t rp, u32 vo, u32 tw4, int s_lo, int s_hi, int s_top,
                                        uint2 (&b)[KaComb<LV>::G][3]) {
  constexpr int G = KaComb<LV>::G;
#pragma unroll
  for (int i = 0; i < G; ++i) {
    if (GI * G + i < KaComb<LV>::NP) {
      const u32 v = vo + (u32)i * tw4;
      b[i][0] = bld8(rp, v, s_lo);
      b[i][1] = bld8(rp, v, s_hi);
      if constexpr (J0) b[i][2] = bld8(rp, v, s_top);
    }
  }
}

// the term table of L levels, evaluated once
template <int LV>
struct KaTab {
  static constexpr KaPoly<LV> P{};
};

// the terms of group g's products, every index a compile-time constant
template <int LV, int GI, int TI, bool J0>
__device__ __forceinline__ void ka_apply_term(i64 (&s)[2 << LV][2], const uint2 (&b)[KaComb<LV>::G][3],
                                              bool hi_half) {
  constexpr KaTerm TT = KaTab<LV>::P.t[TI];
  if constexpr (TT.p / KaComb<LV>::G == GI) {
    // (slabs that land above the entry's 2^(L+1) segments leave it)
    constexpr int i = TT.p - GI * KaComb<LV>::G, NSEG = 2 << LV;
    if constexpr (TT.pw < NSEG) ka_apply(s[TT.pw], b[i][0], TT.sg, false);
    if constexpr (TT.pw + 1 < NSEG) ka_apply(s[TT.pw + 1], b[i][1], TT.sg, false);
    if constexpr (J0 && TT.pw + 2 < NSEG) ka_apply(s[TT.pw + 2], b[i][2], TT.sg, hi_half);
  }
}
template <int LV, int GI, int T0, bool J0, int... I>
__device__ __forceinline__ void ka_apply_group(std::integer_sequence<int, I...>, i64 (&s)[2 << LV][2],
                                               const uint2 (&b)[KaComb<LV>::G][3], bool hi_half) {
  (ka_apply_term<LV, GI, T0 + I, J0>(s, b, hi_half), ...);
}
// the term range of group GI's products (the table is sorted by product)
template <int LV, int GI>
struct KaGroupTerms {
  static constexpr int p0 = GI * KaComb<LV>::G;
  static constexpr int p1 = p0 + KaComb<LV>::G < KaComb<LV>::NP ? p0 + KaComb<LV>::G : KaComb<LV>::NP;
  static constexpr int t0 = KaTab<LV>::P.first[p0], t1 = KaTab<LV>::P.first[p1];
};

// group GI: fence, the loads of group GI + NB - 1, then this group's terms
template <int LV, int GI, bool J0>
__device__ __forceinline__ void ka_group(i64 (&s)[2 << LV][2], KaBuf<LV, J0>& b,
                                         __amdgpu_buffer_rsrc_t rp, u32& vo, u32 tw4, int s_lo, int s_hi, int s_top,
                                         bool hi_half) {
  constexpr int G = KaComb<LV>::G, NG = KaComb<LV>::NG;
  constexpr int NB = KaNb<LV, J0>::NB;
  if constexpr (GI + NB - 1 < NG) {
    // the accumulators after group GI - 1 (whose registers group GI + NB - 1 reuses)
#pragma unroll
    for (int m = 0; m < (2 << LV); m += 2)
      asm volatile("" : "+v"(s[m][0]), "+v"(s[m][1]), "+v"(s[m + 1][0]), "+v"(s[m + 1][1]));
    asm volatile("" : "+v"(vo));
    ka_load<LV, GI + NB - 1, J0>(rp, vo, tw4, s_lo, s_hi, s_top, b[(GI + NB - 1) % NB]);
    vo += (u32)G * tw4;
  }
  using GT = KaGroupTerms<LV, GI>;
  ka_apply_group<LV, GI, GT::t0, J0>(std::make_integer_sequence<int, GT::t1 - GT::t0>{}, s, b[GI % NB],
                                     hi_half);
}
template <int LV, bool J0, int... GI>
__device__ __forceinline__ void ka_groups(std::integer_sequence<int, GI...>, i64 (&s)[2 << LV][2],
                                          KaBuf<LV, J0>& b, __amdgpu_buffer_rsrc_t rp, u32& vo,
                                          u32 tw4, int s_lo, int s_hi, int s_top, bool hi_half) {
  (ka_group<LV, GI, J0>(s, b, rp, vo, tw4, s_lo, s_hi, s_top, hi_half), ...);
}
// the first NB - 1 groups' loads, before any is added in
template <int LV, bool J0, int... GI>
__device__ __forceinline__ void ka_prologue(std::integer_sequence<int, GI...>, KaBuf<LV, J0>& b,
                                            __amdgpu_buffer_rsrc_t rp, u32& vo, u32 tw4, int s_lo, int s_hi,
                                            int s_top) {
  constexpr int G = KaComb<LV>::G, NG = KaComb<LV>::NG;
  ((GI < NG ? (ka_load<LV, (GI < NG ? GI : 0), J0>(rp, vo, tw4, s_lo, s_hi, s_top, b[GI]), vo += (u32)G * tw4)
            : vo), ...);
}

// One slab position jj of every segment: load the segments' slabs, add in the
// terms of every product, resolve the lane pair's carries and store.  J0: jj = 0,
// the only position that also reads the products' top slabs.
template <int LV, bool J0>
__device__ __forceinline__ void ka_slab(int jj, int O, int nq, __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rp,
                                        u32 voff, u32 tw4, bool hi_half, int (&cy)[2 << LV]) {
  constexpr int NSEG = 2 << LV, G = KaComb<LV>::G;
  // The segments' slabs start the accumulators: one 4-byte load per limb
  // straight into the low half of its accumulator, with no branch and no use
  // before the first term, so all of them are in flight at once (the second
  // limb's slab offset goes in the lane offset, which keeps the two loads from
  // being merged into one whose halves would need copies, and waits, to reach
  // the accumulators).  A slab at or above nq reads zero through the
  // descriptor's range check (lane offset past its size).
  i64 s[NSEG][2];
#pragma unroll
  for (int m = 0; m < NSEG; ++m) {
    const int q = m * O + jj;
    const u32 v = q < nq ? voff : kBufferOutOfRange;
    const int so = (q < nq ? q : nq - 1) * 16384;
    s[m][0] = (u32)__builtin_amdgcn_raw_buffer_load_b32(ra, (int)v, so, 0);
    s[m][1] = (u32)__builtin_amdgcn_raw_buffer_load_b32(ra, (int)(v + 4 + (u32)so), 0, 0);
  }
  const int s_lo = jj * 16384, s_hi = (O + jj) * 16384, s_top = 2 * O * 16384;
  KaBuf<LV, J0> b;
  u32 vo = voff;
  ka_prologue<LV, J0>(std::make_integer_sequence<int, KaNb<LV, J0>::NB - 1>{}, b, rp, vo, tw4, s_lo, s_hi, s_top);
  ka_groups<LV, J0>(std::make_integer_sequence<int, KaComb<LV>::NG>{}, s, b, rp, vo, tw4, s_lo, s_hi, s_top,
                    hi_half);
#pragma unroll
  for (int m = 0; m < NSEG; ++m) {
    // limbs 0, 1 with the segment's running carry (low-half lane), their
    // carry into limb 2 to the partner, limbs 2, 3 with it (high-half lane),
    // and the carry out of limb 3 back to the low-half lane (the carries fit
    // 32 bits: a slab sums at most 5^L <= 625 terms of two 32-bit limbs each)
    const i64 a0 = s[m][0] + (hi_half ? 0 : cy[m]);
    const i64 a1 = s[m][1] + (a0 >> 32);
    const int cmid = partner32((int)(a1 >> 32));
    const i64 b0_ = s[m][0] + cmid;
    const i64 b1_ = s[m][1] + (b0_ >> 32);
    const i64 x0 = hi_half ? b0_ : a0, x1 = hi_half ? b1_ : a1;
    cy[m] = partner32((int)(b1_ >> 32));
    if (m * O + jj < nq) {
      const v2u o = {(u32)x0, (u32)x1};
      __builtin_amdgcn_raw_buffer_store_b64(o, ra, (int)voff, (m * O + jj) * 16384, 0);
    }
  }
}

// a -= sum_p c_p(Y) P_p for every live entry of the launch, two lanes per
// entry, in one pass over the 2^(L+1) segments; then the carry out of every
// segment enters at its successor's first slab (the last one leaves the
// entry).  Slabs at or above nq (the entry's nw / 4; there are some when the
// split strings carry zero digits above the factors') read as zero and are not
// written: they only receive carries, and the entry keeps its value modulo
// 2^(32 nw).
template <int LV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LV <= 2 ? 4 : 2)))
void k_kara_comb(KaraArgs k, int C_lo) {
  constexpr int NSEG = 2 << LV;
  const UpdArgs& g = k.m.g;
  const int lt = blockIdx.x >> 3, e = (blockIdx.x & 7) * 128 + (threadIdx.x >> 1);
  const bool hi_half = (threadIdx.x & 1) != 0;
  int R, C;
  // both lanes of a pair see the same entry, so they leave together
  if (!kara_entry(k, C_lo, lt, e, &R, &C) || has_error(g.st)) return;
  const int r = e >> 5, c = e & 31;
  const size_t tix = g.tri ? tri_tile_index(R, C) : (size_t)R * g.ntc + C;
  const size_t tw = tile_words(k.nwp);
  u32* At = g.A + tix * tile_words(g.nw);
  const u32* P0 = k.prod + (size_t)lt * KaComb<LV>::NP * tw;  // this tile's np products
  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(At, 0, (int)(tile_words(g.nw) * 4), kRawBufferWord3);
  const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc(const_cast<u32*>(P0), 0,
                                                                      (int)(KaComb<LV>::NP * tw * 4), kRawBufferWord3);
  const u32 tw4 = (u32)(tw * 4);
  const u32 voff = (u32)in_tile(r, c, 0) * 4 + (hi_half ? 8u : 0u);
  const int O = k.m.S / (16 << LV), nq = g.nw / 4;
  int cy[NSEG];
#pragma unroll
  for (int m = 0; m < NSEG; ++m) cy[m] = 0;
  ka_slab<LV, true>(0, O, nq, ra, rp, voff, tw4, hi_half, cy);
  for (int jj = 1; jj < O; ++jj) ka_slab<LV, false>(jj, O, nq, ra, rp, voff, tw4, hi_half, cy);
  if (!hi_half) {
#pragma unroll
    for (int m = 0; m + 1 < NSEG; ++m) add_at_limb(At, r, c, 4 * (m + 1) * O, g.nw, (i64)cy[m]);
  }
}

// checks of a Karatsuba record against its launch shapes
static bool kara_ok(const KaraArgs& k) {
  const MfmaArgs& m = k.m;
  const UpdArgs& g = m.g;
  const int L = k.levels;
  if (L < 1 || L > KA_MAX_LEVELS || !g.tri || (g.rsb != 0 && g.rsb != (size_t)g.nl)) return false;
  // the split points on whole 4-limb slabs, padding, 32-bit buffer offsets
  bool ok = m.S % (16 << L) == 0 && m.S >= 4 * g.nl && k.Sk == kara_leaf_digits(m.S, L) &&
            k.nwp == kara_nwp(m.S, L) && m.pad >= MF_PAD_MIN && k.kslices == k.Sk + 2 * m.pad &&
            k.nwp / 4 == 2 * (m.S / (16 << L)) + 1;
  for (int l = 1; l <= L; ++l)
    ok = ok && k.pan[l] && k.pan_slices[l] == kara_leaf_digits(m.S, l) + 2 * m.pad &&
         (size_t)k.pan_slices[l] * m.NT * 16 <= 0x7fffffffu && k.pan_stride[l] >= (size_t)k.pan_slices[l] * m.NT * 16;
  return ok;
}

// the digit panels of every level: the factors' halves, their sums, and the
// splits of each level's panels (before the GEMMs)
hipError_t launch_kara_prep(const KaraArgs& k, hipStream_t stream) {
  const MfmaArgs& m = k.m;
  const UpdArgs& g = m.g;
  if (g.r_hi <= g.r_lo || g.c_hi <= g.c_lo || g.npan <= 0) return hipSuccess;
  if (!kara_ok(k)) return hipErrorInvalidValue;
  const int L = k.levels, h = m.S / 2;
  // rows below the launch's first tile row are read by none of its GEMMs
  const int r0 = (g.c_lo / 32) * 32, nr = m.NT - r0;
  const size_t rthreads = (size_t)g.nl * nr * 16;
  const unsigned rblocks = (unsigned)((rthreads + 255) / 256);
  int8_t* l1[6];
  for (int q = 0; q < 6; ++q) l1[q] = k.pan[1] + (size_t)q * k.pan_stride[1];
  hipLaunchKernelGGL(k_recode_kara, dim3(rblocks), dim3(256), 0, stream, g.Bop, g.ldb, g.npan, m.NT, m.NT, g.nl,
                     m.pad, h / 4, l1[0], l1[1], r0);
  hipLaunchKernelGGL(k_recode_kara, dim3(rblocks), dim3(256), 0, stream, g.Uop, g.ldu, g.npan, m.NT, m.u_rows,
                     g.nl, m.pad, h / 4, l1[3], l1[4], r0);
  {
    const size_t threads = (size_t)(h / 4 + 1) * nr;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    hipLaunchKernelGGL(k_kara_mid, dim3(blocks), dim3(256), 0, stream, l1[0], l1[1], m.NT, m.pad, h, l1[2], r0);
    hipLaunchKernelGGL(k_kara_mid, dim3(blocks), dim3(256), 0, stream, l1[3], l1[4], m.NT, m.pad, h, l1[5], r0);
  }
  for (int l = 2; l <= L; ++l) {
    // every level-(l-1) panel (at most S/2^(l-1) + l - 1 digits) splits at S/2^l
    const int nmax = (m.S >> (l - 1)) + l - 1, s = m.S >> l, parents = 2 * kara_products(l - 1);
    const size_t threads = (size_t)nmax * nr;
    hipLaunchKernelGGL(k_digit_split, dim3((unsigned)((threads + 255) / 256), parents), dim3(256), 0, stream, k, l,
                       r0);
    const size_t mthreads = (size_t)((s + l - 1) / 4 + 1) * nr;
    hipLaunchKernelGGL(k_kara_mid_lv, dim3((unsigned)((mthreads + 255) / 256), parents), dim3(256), 0, stream, k, l,
                       r0);
  }
  return hipGetLastError();
}

// the products' range carries, then their combination into the trailing
// matrix (after the GEMMs of a launch of ntiles tiles from tile row C_lo)
hipError_t launch_kara_finish(const KaraArgs& k, const RangeTab& rt, int C_lo, int ntiles, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  const int L = k.levels, np = kara_products(L);
  if (rt.n > 1) hipLaunchKernelGGL(k_kara_fix, dim3(4 * ntiles, np), dim3(256), 0, stream, k, rt, C_lo, ntiles);
  // two lanes per entry: 8 blocks of 256 threads per tile
  if (L == 1)
    hipLaunchKernelGGL(k_kara_comb<1>, dim3(8 * ntiles), dim3(256), 0, stream, k, C_lo);
  else if (L == 2)
    hipLaunchKernelGGL(k_kara_comb<2>, dim3(8 * ntiles), dim3(256), 0, stream, k, C_lo);
  else if (L == 3)
    hipLaunchKernelGGL(k_kara_comb<3>, dim3(8 * ntiles), dim3(256), 0, stream, k, C_lo);
  else
    hipLaunchKernelGGL(k_kara_comb<4>, dim3(8 * ntiles), dim3(256), 0, stream, k, C_lo);
  return hipGetLastError();
}

hipError_t launch_upd_kara(const KaraArgs& k, hipStream_t stream) {
  const MfmaArgs& m = k.m;
  const UpdArgs& g = m.g;
  if (g.r_hi <= g.r_lo || g.c_hi <= g.c_lo || g.npan <= 0) return hipSuccess;
  hipError_t e = launch_kara_prep(k, stream);
  if (e != hipSuccess) return e;
  const int np = kara_products(k.levels);
  const int nt = m.NT / 32;
  const int C_lo = g.c_lo / 32;
  const int ncol = nt - C_lo;
  const int ntiles = ncol * (ncol + 1) / 2;
  if ((size_t)ntiles > k.prod_tiles) return hipErrorInvalidValue;
  const RangeTab rt = make_ranges_ntb(k.nwp / 4, k.Sk, (long)np * ntiles, m.max_ranges, m.carry_tiles);
  if ((size_t)np * ntiles * rt.n > m.carry_tiles) return hipErrorInvalidValue;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (m.timing) {
    (void)hipEventCreate(&ev0);
    (void)hipEventCreate(&ev1);
    (void)hipEventRecord(ev0, stream);
  }
  const long items = (long)np * ntiles * rt.n;
  const int per_xcd = (int)((items + 7) / 8);
  e = launch_kara_gemm(k, rt, C_lo, ntiles, per_xcd, stream);
  if (m.timing) {
    (void)hipEventRecord(ev1, stream);
    (void)hipEventSynchronize(ev1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ev0, ev1);
    m.timing->ms[6] += ms;
    m.timing->launches[1] += 1;
    m.timing->launches[2] += 1;
    m.timing->launches[3] += k.levels;
    (void)hipEventRecord(ev0, stream);
  }
  if (e != hipSuccess) return e;
  e = launch_kara_finish(k, rt, C_lo, ntiles, stream);
  if (m.timing) {
    (void)hipEventRecord(ev1, stream);
    (void)hipEventSynchronize(ev1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ev0, ev1);
    m.timing->ms[9] += ms;
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
  }
  return e;
}

}  // namespace hl
