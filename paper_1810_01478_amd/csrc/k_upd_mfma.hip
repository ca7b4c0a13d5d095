// Exact Schur-complement update as int8 MFMA GEMMs (the "slice" form):
//   A[r][c] <- A[r][c] - sum_{i in panel} b_ri u_ci        (Algorithm 1, inner loops)
//
// Digits.  Each P-bit two's complement factor x is recoded into S = P/8 signed
// base-256 digits in [-128, 127], x = sum_j x_j 256^j (the bound
// |x| < 3 2^(P-3) keeps the top digit in range).  Then
//   sum_i b_ri u_ci = sum_t 256^t out_t(r, c),
//   out_t(r, c) = sum_j sum_i beta_{r,i,j} upsilon_{c,i,t-j},
// which for each output digit t is an exact int8 GEMM over K = (i, j) with
// int32 accumulation (16 panel columns x up to S digits x 2^14 < 2^31 for
// S <= 8191).  The second operand is a Toeplitz matrix in (t, j).
//
// Kernel.  One wave owns a 32 x 32 tile of the trailing matrix and a range of
// output limbs.  v_mfma_i32_32x32x32_i8 takes K = 32 = 2 digits x 16 panel
// columns: lane half h of the A operand holds the 16 panel columns of digit
// j0 + h for row m; of the B operand, digit t - j0 - h for column n.  Output
// digits are taken 16 at a time (16 accumulators of 16 registers, one 4-limb
// slab of each entry); for the 16 accumulators of one step the B operands are
// 16 consecutive digit slices, and the next step (j0 + 2) needs the same slices
// shifted by two, so a window of 20 slices rotates through registers: each step
// loads one A slice and two B slices for the step after next and issues 16
// MFMAs, 3 KiB of operands per 2^19 int8 multiply-adds.  Digit slices outside
// [0, S) are zero padding.  One wave per SIMD (the accumulators fill the
// accumulation registers); the work items are grouped per XCD so that the waves
// resident on one XCD stream the same slices through its L2.
//
// Recombination.  After the j loop of 16 output digits (4 limbs), each lane folds
// its 16 entries: X = A[2 limbs] - sum_q out_(t0+q) 256^q + carry, an exact
// 128-bit value, twice; the low 64 bits are the new limbs and X >> 64 the carry
// into the next pair of limbs.  The carry out of each wave's limb range is
// stored and added by k_carry_fix, so ranges of one tile run in parallel.
#include <type_traits>
#include <utility>

#include "hl_kernels.hpp"

namespace hl {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// the tile loop's constants (MF_T, MF_PF, MF_WIN, MF_ROT, MF_PAD_MIN) are in hl_kernels.hpp

// entry (m, n) of the 32 x 32 MFMA result held by lane l, register v
__device__ __forceinline__ int mf_row(int l, int v) { return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3); }
__device__ __forceinline__ int mf_col(int l) { return l & 31; }

// ---------------------------------------------------------------------------
// Recode the panel factors (two's complement, nl limbs) into balanced digits.
// src: [16][NT][nl] limbs; dst: [slices][NT][16] bytes, slice = digit + pad.
// One thread per (limb q, row, panel column): digits 4q .. 4q+3.
__device__ __forceinline__ void recode_body(const u32* __restrict__ src, size_t lds, int npan, int NT, int nrows,
                                            int nl, int pad, int8_t* __restrict__ dst, size_t gid) {
  const int il = (int)(gid & 15);
  const size_t t = gid >> 4;
  const int row = (int)(t % NT), q = (int)(t / NT);
  if (q >= nl) return;
  const size_t rstride = (size_t)NT * 16;
  int8_t* d = dst + (size_t)(pad + 4 * q) * rstride + (size_t)row * 16 + il;
  u32 v = 0;
  if (il < npan && row < nrows) v = balanced_digits4(src + (size_t)il * lds + (size_t)row * nl, nl, q);
#pragma unroll
  for (int b = 0; b < 4; ++b) d[(size_t)b * rstride] = (int8_t)(v >> (8 * b));
}

__global__ void k_recode(const u32* __restrict__ src, size_t lds, int npan, int NT, int nrows, int nl, int pad,
                         int8_t* __restrict__ dst) {
  recode_body(src, lds, npan, NT, nrows, nl, pad, dst, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// batch: blockIdx.y is the record
__global__ void k_recode_b(const RecodeArgs* __restrict__ tab) {
  const RecodeArgs& a = tab[blockIdx.y];
  recode_body(a.src, a.lds, a.npan, a.NT, a.nrows, a.nl, a.pad, a.dst, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__device__ __forceinline__ v4i ld16(const int8_t* p) { return *(const v4i*)p; }

// 16 bytes at byte offset voff (per lane) + soff (wave-uniform) of a buffer
__device__ __forceinline__ v4i bld16(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
}

// s_waitcnt immediate for vmcnt(0) with expcnt and lgkmcnt left at their
// maxima (gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int kVmcntZero = 0x0F70;

// index of tile (R, C) among the tiles of one launch, for its carry slots
__device__ __forceinline__ size_t launch_tile_index(const UpdArgs& g, int R, int C, int C_lo) {
  if (g.tri) {
    const size_t r = R - C_lo;
    return r * (r + 1) / 2 + (C - C_lo);
  }
  return (size_t)(R - C_lo) * g.ntc + C;
}

// The digit-sum GEMM of tile (R, C) over output blocks [tb0, tb1) of the
// product of the digit panels bdig (rows) and udig (columns), S digits each,
// slices = S + 2 pad slices of NT x 16 bytes.  STORE = false: the sums are
// subtracted from the trailing-matrix tile Out (limb 4 tb of an entry receives
// block tb).  STORE = true: the exact sums themselves are written to the tile
// Out, block tb as limbs 4 tb .. 4 tb + 3 of the entry.  Either way the carry
// out of the range goes to cb (1024 entries).
// acc * m2 + d for an int32 digit sum acc and m2 = 2^(8 m): one 32 x 32 ->
// 64-bit signed multiply-add (v_mad_i64_i32) once m2 is opaque to the compiler
// (a known power of two would become 64-bit shifts)
__device__ __forceinline__ i64 mad_digit(int acc, int m2, i64 d) { return (i64)acc * (i64)m2 + d; }
// one accumulator register, read from the accumulation file by itself (an
// element taken from the vector otherwise copies the whole vector)
__device__ __forceinline__ int acc_elem(int a) {
  int v;
  asm("v_accvgpr_read_b32 %0, %1" : "=v"(v) : "a"(a));
  return v;
}
__device__ __forceinline__ int opaque_i32(int v) {
  asm volatile("" : "+s"(v));
  return v;
}

// The digit-sum GEMM of tile (R, C) over output blocks [tb0, tb1) of the
// product of the digit panels bdig (rows) and udig (columns), S digits each,
// slices = S + 2 pad slices of NT x 16 bytes.  STORE = false: the sums are
// subtracted from the trailing-matrix tile Out (limb 4 tb of an entry receives
// block tb).  STORE = true: the exact sums themselves are written to the tile
// Out, block tb as limbs 4 tb .. 4 tb + 3 of the entry.  Either way the carry
// out of the range goes to cb (1024 entries).
//
// Per block the steps run in whole rotations of the register window and one
// last partial rotation whose steps are skipped past the block's end (no
// padding steps); the next block's operands are requested before this block's
// sums are folded, so their latency hides behind the fold.
// MFMAs a step issues: all MF_T, or in the first rotation of a skipping
// block those whose digit pairs reach an output digit (see mfma_tile_t)
constexpr int mf_issued(int st, bool skip, bool rev) {
  int n = 0;
  for (int q = 0; q < MF_T; ++q)
    if (!skip || (rev ? q >= MF_T - 2 - 2 * st : q <= 2 * st + 1)) ++n;
  return n;
}

// f(integral_constant<int, 0>) .. f(integral_constant<int, N - 1>), in order
template <typename F, int... I>
__device__ __forceinline__ void mf_unroll_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void mf_unroll(F&& f) {
  mf_unroll_seq(f, std::make_integer_sequence<int, N>{});
}

constexpr int MF_FOLD = 4;  // entries folded together

template <bool STORE>
__device__ __forceinline__ void mfma_tile_t(const UpdArgs& g, const int8_t* bdig, const int8_t* udig, int slices,
                                            int S, int pad, int NT, int R, int C, int tb0, int tb1, long long* cb,
                                            u32* Out, int out_nw) {
  if (has_error(g.st)) return;
  __shared__ int carry_s[16 * WAVE];  // carry of each of the lane's 16 entries (|carry| < 2^25)
  const int l = lane_id(), h = l >> 5, mm = l & 31;
  const int sst = NT * 16;  // bytes per digit slice
  // A operand (b digits of tile rows), B operand (u digits of tile columns),
  // read through buffer descriptors: a 32-bit lane offset plus a wave-uniform
  // slice offset stepped in scalar registers, so no load in flight holds a
  // per-lane 64-bit address; loads past the panels return zero
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<int8_t*>(bdig), 0, slices * sst, kRawBufferWord3);
  const __amdgpu_buffer_rsrc_t ru =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<int8_t*>(udig), 0, slices * sst, kRawBufferWord3);
  // the output tile: entry (r, c) of slab tb at byte 16 (1024 tb + 32 r + c);
  // the lane's part of that offset in a register, the slab's and the
  // accumulator register's in a scalar one
  const __amdgpu_buffer_rsrc_t ro =
      __builtin_amdgcn_make_buffer_rsrc(Out, 0, (int)(tile_words(out_nw) * 4), kRawBufferWord3);
  const int ooff = (4 * h * 32 + mm) * 16;
  const int aoff = h * sst + R * 512 + mm * 16;
  const int uoff = (1 - h) * sst + C * 512 + mm * 16;
  unsigned live = 0;  // entries of the trailing matrix proper (r >= c, inside the target)
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    carry_s[v * WAVE + l] = 0;
    const int r = R * 32 + mf_row(l, v), c = C * 32 + mf_col(l);
    if ((!g.tri || r >= c) && r >= g.r_lo && r < g.r_hi && c >= g.c_lo && c < g.c_hi) live |= 1u << v;
  }
  // The steps of a block are the digit pairs (j, j + 1), j = jlo, jlo + 2, ..,
  // jtop; forward blocks take them upwards, reverse blocks downwards (the same
  // pairs, so the same sums).  Forward: window slot (y mod MF_WIN) holds the
  // u slice at digit t0 - jlo + y (minus the lane half); step s multiplies
  // y = q - 2s for q = 0..MF_T-1 and loads y = -2 MF_PF - 2s, -2 MF_PF + 1 - 2s
  // for step s + MF_PF.  Reverse: slot y holds digit t0 - jtop + y; step r
  // multiplies y = q + 2r and loads y = 2 MF_PF + 2r + 14, + 15.  A digits are
  // loaded MF_PF steps ahead into a ring either way.
  //
  // Output digit t0 + q gets nothing from pair j when t0 + q - j - 1 > S - 1 or
  // t0 + q - j < 0.  A block with t0 >= S - 1 has jlo >= t0 - S, so its first
  // steps s = 0..7 (forward) need only q <= 2s + 1; a block with
  // t0 + MF_T - 1 <= S - 1 has jtop = t0 + 14, so its first steps r = 0..6
  // (reverse) need only q >= 14 - 2r.  Those blocks run their first rotation
  // with the other MFMAs left out (at compile time); the block between the two
  // kinds runs forward with all of them.
  v4i w[MF_WIN];
  v4i an[MF_PF];
  int ap = 0, un = 0, nsteps = 0, dir = 0;  // dir: 0 forward, 1 forward skipping, 2 reverse skipping
  // block tb's steps and its first operands (REV: a block of the first kind
  // below, run downwards)
  auto prologue = [&](int tb_, auto revc) {
    constexpr bool REV = decltype(revc)::value;
    const int t0_ = MF_T * tb_;
    int jlo_ = t0_ - (S - 1);
    if (jlo_ < 0) jlo_ = 0;
    jlo_ &= ~1;
    int jhi_ = t0_ + MF_T - 1;
    if (jhi_ > S - 1) jhi_ = S - 1;
    nsteps = (jhi_ - jlo_) / 2 + 1;
    if (!REV) {
      dir = t0_ >= S - 1 ? 1 : 0;
      const int ub_ = (pad - 1 + t0_ - jlo_) * sst;
#pragma unroll
      for (int y = 0; y < MF_T; ++y) w[y] = bld16(ru, uoff, ub_ + y * sst);
#pragma unroll
      for (int y = -2 * (MF_PF - 1); y < 0; ++y) w[MF_WIN + y] = bld16(ru, uoff, ub_ + y * sst);
      ap = (pad + jlo_) * sst;
#pragma unroll
      for (int q = 0; q < MF_PF; ++q) an[q] = bld16(rb, aoff, ap + 2 * q * sst);
      ap += 2 * MF_PF * sst;
      un = ub_ - 2 * MF_PF * sst;
    } else {
      dir = 2;
      const int jtop_ = jlo_ + 2 * (nsteps - 1);
      const int ub_ = (pad - 1 + t0_ - jtop_) * sst;
#pragma unroll
      for (int y = 0; y < MF_T + 2 * (MF_PF - 1); ++y) w[y] = bld16(ru, uoff, ub_ + y * sst);
      ap = (pad + jtop_) * sst;
#pragma unroll
      for (int q = 0; q < MF_PF; ++q) an[q] = bld16(rb, aoff, ap - 2 * q * sst);
      ap -= 2 * MF_PF * sst;
      un = ub_ + (MF_T + 2 * (MF_PF - 1)) * sst;
    }
  };
  v16i acc[MF_T];
  // one step (its place st in the rotation and the skip, compile-time constants)
  auto step_f = [&](auto stc, auto skc) {
    constexpr int st = decltype(stc)::value;
    constexpr bool SK = decltype(skc)::value;
    const v4i a_ = an[st % MF_PF];
    an[st % MF_PF] = bld16(rb, aoff, ap);
    constexpr int k0 = (MF_WIN * 4 - 2 * MF_PF - 2 * st) % MF_WIN;
    w[k0] = bld16(ru, uoff, un);
    w[k0 + 1] = bld16(ru, uoff, un + sst);
#pragma unroll
    for (int q = 0; q < MF_T; ++q)
      if (!SK || q <= 2 * st + 1)
        acc[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a_, w[(q - 2 * st + MF_WIN * 4) % MF_WIN], acc[q], 0, 0, 0);
    ap += 2 * sst;
    un -= 2 * sst;
    __builtin_amdgcn_sched_group_barrier(0x020, 3, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, mf_issued(st, SK, false), 0);
  };
  auto step_r = [&](auto stc, auto skc) {
    constexpr int st = decltype(stc)::value;
    constexpr bool SK = decltype(skc)::value;
    const v4i a_ = an[st % MF_PF];
    an[st % MF_PF] = bld16(rb, aoff, ap);
    constexpr int k0 = (2 * st + MF_T + 2 * (MF_PF - 1)) % MF_WIN;
    w[k0] = bld16(ru, uoff, un);
    w[k0 + 1] = bld16(ru, uoff, un + sst);
#pragma unroll
    for (int q = 0; q < MF_T; ++q)
      if (!SK || q >= MF_T - 2 - 2 * st)
        acc[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a_, w[(q + 2 * st) % MF_WIN], acc[q], 0, 0, 0);
    ap -= 2 * sst;
    un += 2 * sst;
    __builtin_amdgcn_sched_group_barrier(0x020, 3, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, mf_issued(st, SK, true), 0);
  };
  using SkipOn = std::integral_constant<bool, true>;
  using SkipOff = std::integral_constant<bool, false>;

  auto fold = [&](int tb) {
    // fold the 16 digit sums of each entry into limbs 4 tb .. 4 tb + 3 (one
    // slab): V = sum_k d_k 2^(32 k) + carry, d_k = sum_m out_(t0+4k+m) 2^(8 m)
    // (|d_k| < 2^56, exact in 64 bits), resolved 32 bits at a time: t_0 = d_0 +
    // carry, t_k = d_k + (t_(k-1) >> 32); the limbs are the low halves of t_k
    // (or of the old limbs minus d_k plus the carry), the carry t_3 >> 32.
    // Every step is one 32 x 32 -> 64-bit signed multiply-add (the multipliers
    // are opaque, the carry enters with multiplier 1).  A product tile (STORE)
    // is written whole, dead entries included: nothing reads them.
    const int m8 = opaque_i32(1 << 8), m16 = opaque_i32(1 << 16), m24 = opaque_i32(1 << 24);
    const int one = opaque_i32(1);
    const int soff_tb = tb * (MF_LPB * 4096);
    // four entries at a time, so that their independent chains interleave
#pragma unroll
    for (int v0 = 0; v0 < 16; v0 += MF_FOLD) {
      i64 t[MF_FOLD][4];
#pragma unroll
      for (int e = 0; e < MF_FOLD; ++e) {
        const int v = v0 + e;
        if (STORE) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            i64 x = (i64)acc_elem(acc[4 * k][v]);
            x = mad_digit(acc_elem(acc[4 * k + 1][v]), m8, x);
            x = mad_digit(acc_elem(acc[4 * k + 2][v]), m16, x);
            t[e][k] = mad_digit(acc_elem(acc[4 * k + 3][v]), m24, x);
          }
        } else {
          if (!((live >> v) & 1u)) continue;
          const int soff = soff_tb + (8 * (v >> 2) + (v & 3)) * 512;
          const v4i x = __builtin_amdgcn_raw_buffer_load_b128(ro, ooff, soff, 0);
          const int n1 = opaque_i32(-1), n8 = opaque_i32(-(1 << 8)), n16 = opaque_i32(-(1 << 16)),
                    n24 = opaque_i32(-(1 << 24));
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            i64 y = (i64)(u32)x[k];
            y = mad_digit(acc_elem(acc[4 * k][v]), n1, y);
            y = mad_digit(acc_elem(acc[4 * k + 1][v]), n8, y);
            y = mad_digit(acc_elem(acc[4 * k + 2][v]), n16, y);
            t[e][k] = mad_digit(acc_elem(acc[4 * k + 3][v]), n24, y);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < MF_FOLD; ++e) {
        const int v = v0 + e;
        if (!STORE && !((live >> v) & 1u)) continue;
        t[e][0] = mad_digit(carry_s[v * WAVE + l], one, t[e][0]);
      }
#pragma unroll
      for (int k = 1; k < 4; ++k) {
#pragma unroll
        for (int e = 0; e < MF_FOLD; ++e) t[e][k] = mad_digit((int)(t[e][k - 1] >> 32), one, t[e][k]);
      }
#pragma unroll
      for (int e = 0; e < MF_FOLD; ++e) {
        const int v = v0 + e;
        if (!STORE && !((live >> v) & 1u)) continue;
        const int soff = soff_tb + (8 * (v >> 2) + (v & 3)) * 512;
        const v4i o = {(int)(u32)t[e][0], (int)(u32)t[e][1], (int)(u32)t[e][2], (int)(u32)t[e][3]};
        __builtin_amdgcn_raw_buffer_store_b128(o, ro, ooff, soff, 0);
        carry_s[v * WAVE + l] = (int)(t[e][3] >> 32);
      }
    }
  };
  // blocks [ta, te) of one kind, each its steps and then its fold
  auto run_blocks = [&](int ta, int te, auto revc) {
    constexpr bool REV = decltype(revc)::value;
    if (ta >= te) return;
    prologue(ta, revc);
    for (int tb = ta; tb < te; ++tb) {
#pragma unroll
      for (int q = 0; q < MF_T; ++q) acc[q] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      // Let the prologue's loads land here, once per block: the loop header
      // then only sees the loads in flight from the previous rotation, and its
      // wait keeps the MF_PF steps of prefetch instead of draining them every
      // rotation.
      __builtin_amdgcn_s_waitcnt(kVmcntZero);
      // the first rotation of a skipping block (steps past the block's end
      // left out), then whole rotations, then one partial rotation
      int left = nsteps;
      if (REV) {
        mf_unroll<MF_ROT>([&](auto stc) {
          if (decltype(stc)::value < left) step_r(stc, SkipOn{});
        });
        left -= MF_ROT;
        for (; left >= MF_ROT; left -= MF_ROT) mf_unroll<MF_ROT>([&](auto stc) { step_r(stc, SkipOff{}); });
        mf_unroll<MF_ROT - 1>([&](auto stc) {
          if (decltype(stc)::value < left) step_r(stc, SkipOff{});
        });
      } else {
        if (dir == 1) {
          mf_unroll<MF_ROT>([&](auto stc) {
            if (decltype(stc)::value < left) step_f(stc, SkipOn{});
          });
          left -= MF_ROT;
        }
        for (; left >= MF_ROT; left -= MF_ROT) mf_unroll<MF_ROT>([&](auto stc) { step_f(stc, SkipOff{}); });
        mf_unroll<MF_ROT - 1>([&](auto stc) {
          if (decltype(stc)::value < left) step_f(stc, SkipOff{});
        });
      }
      // the next block's first operands, in flight during the fold
      if (tb + 1 < te) prologue(tb + 1, revc);
      fold(tb);
    }
  };
  // blocks with t0 + MF_T - 1 <= S - 1 run downwards, the others upwards; the
  // two loops share no registers, so each keeps its own window in place
  const int tb_rev = S >= MF_T ? (S - MF_T) / MF_T + 1 : 0;
  run_blocks(tb0, tb1 < tb_rev ? tb1 : tb_rev, std::integral_constant<bool, true>{});
  run_blocks(tb0 > tb_rev ? tb0 : tb_rev, tb1, std::integral_constant<bool, false>{});
  // carries out of this range
#pragma unroll
  for (int v = 0; v < 16; ++v) cb[mf_row(l, v) * 32 + mf_col(l)] = (long long)carry_s[v * WAVE + l];
}

// the Schur update of tile (R, C) of the trailing matrix (see mfma_tile_t)
__device__ __forceinline__ void mfma_tile(const MfmaArgs& m, int R, int C, int tb0, int tb1, long long* cb) {
  const UpdArgs& g = m.g;
  const size_t tix = g.tri ? tri_tile_index(R, C) : (size_t)R * g.ntc + C;
  mfma_tile_t<false>(g, m.bdig, m.udig, m.slices, m.S, m.pad, m.NT, R, C, tb0, tb1, cb,
                     g.A + tix * tile_words(g.nw), g.nw);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_upd_mfma(MfmaArgs m, RangeTab rt, int C_lo, int ntiles, int per_xcd) {
  const UpdArgs& g = m.g;
  // Work items (range rg, tile lt) in range-major order; the workgroups of a
  // launch are dealt to the 8 XCDs in turn, so block b takes item
  // (b % 8) * per_xcd + b / 8: the waves resident on one XCD share a limb range
  // and hold neighbouring tiles, and read the same digit slices from its L2.
  const int b = blockIdx.x;
  const int item = (b & 7) * per_xcd + (b >> 3);
  if (item >= ntiles * rt.n) return;
  const int rg = item / ntiles, lt = item - rg * ntiles;
  // triangular target: tiles (R, C), C_lo <= C <= R, row by row; rectangular:
  // tile rows from C_lo (here the first tile row), all g.ntc tile columns
  int R, C;
  item_tile(g, C_lo, lt, &R, &C);
  if (R * 32 >= m.NT) return;
  mfma_tile(m, R, C, rt.tb[rg], rt.tb[rg + 1], m.carry + ((size_t)lt * rt.n + rg) * 1024);
}

// The batch kernel's two kinds of work item, each its own function: inlined
// together, the two tile loops would share one register allocation and spill.
__device__ __noinline__ void batch_tile_store(const MfmaEntry& e, int R, int C, int lt, int rg, long long* cb) {
  mfma_tile_t<true>(e.m.g, e.m.bdig, e.m.udig, e.m.slices, e.m.S, e.m.pad, e.m.NT, R, C, e.rt.tb[rg], e.rt.tb[rg + 1],
                    cb, e.store + (size_t)lt * e.store_ts, e.store_nw);
}
__device__ __noinline__ void batch_tile_sub(const MfmaEntry& e, int R, int C, int rg, long long* cb) {
  mfma_tile(e.m, R, C, e.rt.tb[rg], e.rt.tb[rg + 1], cb);
}

// Batch of updates (one entry per instance, or per Karatsuba product of an
// instance) in one persistent launch.  Work items (entry, tile, range) sit in 8
// queues, one per XCD, each largest first;
// a wave takes the next item of its XCD's queue until the queue is empty (every
// wave reaches that exit: the queues are finite and nothing waits on another
// wave).  heads[8] must be zero at launch.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_upd_mfma_b(const MfmaEntry* __restrict__ tab, const int4* __restrict__ items, int per_xcd,
                  unsigned* __restrict__ heads) {
  const int xcd = blockIdx.x & 7;
  for (;;) {
    int k = 0;
    if (lane_id() == 0) k = (int)atomicAdd(heads + xcd, 1u);
    k = __shfl(k, 0, WAVE);
    if (k >= per_xcd) break;
    const int4 it = items[(size_t)xcd * per_xcd + k];
    if (it.x < 0) continue;
    const MfmaEntry& e = tab[it.x];
    int R, C;
    item_tile(e.m.g, e.C_lo, it.y, &R, &C);
    if (R * 32 >= e.m.NT) continue;
    long long* cb = e.m.carry + ((size_t)it.y * e.rt.n + it.z) * 1024;
    if (e.store)
      batch_tile_store(e, R, C, it.y, it.z, cb);
    else
      batch_tile_sub(e, R, C, it.z, cb);
  }
}

// Add the carries of range w at limb MF_LPB tb[w+1] of every entry, w = 0..n-2.
__device__ __forceinline__ void carry_fix_body(const MfmaArgs& m, const RangeTab& rt, int C_lo, int bx, int by) {
  const UpdArgs& g = m.g;
  const int R = C_lo + bx, C = g.tri ? C_lo + by : by;
  if ((g.tri && R < C) || R * 32 >= m.NT || (!g.tri && C >= g.ntc)) return;
  if (has_error(g.st)) return;
  const size_t tix = g.tri ? tri_tile_index(R, C) : (size_t)R * g.ntc + C;
  const int e = threadIdx.x;  // 0..1023
  const int r = e >> 5, c = e & 31;
  {
    const int rg = R * 32 + r, cg = C * 32 + c;
    if (!((!g.tri || rg >= cg) && rg >= g.r_lo && rg < g.r_hi && cg >= g.c_lo && cg < g.c_hi)) return;
  }
  u32* At = g.A + tix * tile_words(g.nw);
  const long long* cb = m.carry + launch_tile_index(g, R, C, C_lo) * rt.n * 1024;
  const int nw = m.g.nw;
  for (int w = 0; w + 1 < rt.n; ++w) {
    const i64 cv = cb[(size_t)w * 1024 + e];
    if (cv == 0) continue;
    int li = MF_LPB * rt.tb[w + 1];
    if (li >= nw) continue;
    // add the sign-extended 64-bit value cv at limb li
    u32* p0 = At + in_tile(r, c, li);
    u64 a = ((u64)p0[1] << 32) | p0[0];
    u64 s2 = a + (u64)cv;
    u64 cy = s2 < a ? 1 : 0;
    p0[0] = (u32)s2;
    p0[1] = (u32)(s2 >> 32);
    // higher limbs receive (cv < 0 ? -1 : 0) + cy
    const u64 add = (cv < 0 ? ~0ull : 0ull) + cy;  // 0 (done), 1 (carry) or ~0 (borrow)
    if (add == 0) continue;
    for (li += 2; li < nw; li += 2) {
      u32* p = At + in_tile(r, c, li);
      const u64 x = ((u64)p[1] << 32) | p[0];
      const u64 y = x + add;
      p[0] = (u32)y;
      p[1] = (u32)(y >> 32);
      // continue while the carry or borrow runs on
      if (add == 1 ? (y != 0) : (x != 0)) break;
    }
  }
}

__global__ void k_carry_fix(MfmaArgs m, RangeTab rt, int C_lo) { carry_fix_body(m, rt, C_lo, blockIdx.x, blockIdx.y); }

// batch: blockIdx.z is the entry
__global__ void k_carry_fix_b(const MfmaEntry* __restrict__ tab) {
  const MfmaEntry& e = tab[blockIdx.z];
  if (e.rt.n > 1 && !e.store) carry_fix_body(e.m, e.rt, e.C_lo, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Karatsuba form (see KaraArgs; recodes, splits and the recombination are in
// k_kara.hip).  The digit-sum GEMMs of the products: work items (range rg,
// product p, tile lt) in that order, dealt to the XCDs as in k_upd_mfma, so the waves of one
// XCD share a range and a product and hold neighbouring tiles.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_upd_kara(KaraArgs k, RangeTab rt, int C_lo, int ntiles, int per_xcd) {
  const UpdArgs& g = k.m.g;
  const int np = kara_products(k.levels);
  const int b = blockIdx.x;
  const int item = (b & 7) * per_xcd + (b >> 3);
  if (item >= np * ntiles * rt.n) return;
  const int rg = item / (np * ntiles), rem = item - rg * np * ntiles;
  const int p = rem / ntiles, lt = rem - p * ntiles;
  int R, C;
  item_tile(g, C_lo, lt, &R, &C);
  if (R * 32 >= k.m.NT) return;
  const int8_t* leaf = k.pan[k.levels];
  const size_t ls = k.pan_stride[k.levels];
  // the product's own operand length: the steps and blocks past it are empty
  mfma_tile_t<true>(g, leaf + (size_t)p * ls, leaf + (size_t)(np + p) * ls, k.kslices,
                    kara_prod_digits(k.m.S, k.levels, p), k.m.pad, k.m.NT, R, C, rt.tb[rg], rt.tb[rg + 1],
                    k.m.carry + (((size_t)p * ntiles + lt) * rt.n + rg) * 1024,
                    k.prod + ((size_t)lt * np + p) * tile_words(k.nwp), k.nwp);
}

// ---------------------------------------------------------------------------
// MFMA output layout probe (test hook): out[v * 64 + l] for two operand patterns.
__global__ __launch_bounds__(64) void k_mfma_probe(int* out) {
  const int l = lane_id();
  const int8_t am = (int8_t)((l & 31) + 1);
  v4i a1, b1, a2, b2;
  int8_t* pa1 = (int8_t*)&a1;
  int8_t* pb1 = (int8_t*)&b1;
  int8_t* pa2 = (int8_t*)&a2;
  int8_t* pb2 = (int8_t*)&b2;
  for (int i = 0; i < 16; ++i) {
    pa1[i] = am;
    pb1[i] = 1;
    pa2[i] = 1;
    pb2[i] = am;
  }
  v16i z = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  v16i d1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, z, 0, 0, 0);
  v16i d2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, b2, z, 0, 0, 0);
  for (int v = 0; v < 16; ++v) {
    out[v * 64 + l] = d1[v];
    out[1024 + v * 64 + l] = d2[v];
  }
}

// ---------------------------------------------------------------------------
// Digit-pair work of output block tb (the (t, j) pairs it multiplies).
double block_work(int tb, int S) {
  double w = 0;
  for (int q = 0; q < MF_T; ++q) {
    const int t = MF_T * tb + q;
    int cnt = t + 1;
    if (cnt > S) cnt = S;
    if (2 * S - 1 - t < cnt) cnt = 2 * S - 1 - t;
    if (cnt > 0) w += cnt;
  }
  return w;
}

// Split the output blocks of every tile into ranges of about equal work.  The
// number of ranges minimises the launch's time in units of one tile's work,
// rounds x (1/n + c), where one round is one wave on each of the 1024 SIMDs
// (8 XCDs x 128) and c = 0.2% of a tile is the cost of one more work item (its
// first block's operand fetch and its carry slot).
RangeTab make_ranges(int nl, int S, int ntiles, int max_ranges, size_t max_items) {
  return make_ranges_ntb(8 * nl / MF_T, S, ntiles, max_ranges, max_items);
}

RangeTab make_ranges_ntb(int ntb, int S, long units, int max_ranges, size_t max_items) {
  int cap = max_ranges < MF_MAX_RANGES ? max_ranges : MF_MAX_RANGES;
  if (cap > ntb) cap = ntb;
  if (cap < 1) cap = 1;
  int want = 1;
  double best = 1e300;
  for (int n = 1; n <= cap; ++n) {
    const long total = units * n;
    if (n > 1 && (size_t)total > max_items) break;
    const long per = (total + 7) / 8;
    const long rounds = (per + 127) / 128;
    const double cost = (double)rounds * (1.0 / n + 0.002);
    if (cost < best * 0.999) {
      best = cost;
      want = n;
    }
  }
  return split_ranges_ntb(ntb, S, want);
}

// n ranges of about equal work
RangeTab split_ranges(int nl, int S, int want) { return split_ranges_ntb(8 * nl / MF_T, S, want); }

RangeTab split_ranges_ntb(int ntb, int S, int want) {
  RangeTab rt{};
  if (want < 1) want = 1;
  if (want > MF_MAX_RANGES) want = MF_MAX_RANGES;
  if (want > ntb) want = ntb;
  double total = 0;
  for (int tb = 0; tb < ntb; ++tb) total += block_work(tb, S);
  rt.tb[0] = 0;
  double acc = 0;
  int k = 1;
  for (int tb = 0; tb < ntb && k < want; ++tb) {
    acc += block_work(tb, S);
    if (acc >= total * k / want) rt.tb[k++] = tb + 1;
  }
  while (k < want) rt.tb[k++] = ntb;
  rt.tb[want] = ntb;
  // drop empty ranges
  int w = 1;
  for (int j = 1; j <= want; ++j)
    if (rt.tb[j] > rt.tb[w - 1]) rt.tb[w++] = rt.tb[j];
  rt.n = w - 1;
  return rt;
}

hipError_t launch_recode(const u32* src, size_t lds, int npan, int NT, int nrows, int nl, int pad, int8_t* dst,
                         hipStream_t stream) {
  const size_t threads = (size_t)nl * NT * 16;
  hipLaunchKernelGGL(k_recode, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, stream, src, lds, npan, NT,
                     nrows, nl, pad, dst);
  return hipGetLastError();
}

hipError_t launch_upd_mfma(const MfmaArgs& m, hipStream_t stream) {
  const UpdArgs& g = m.g;
  if (g.r_hi <= g.r_lo || g.c_hi <= g.c_lo || g.npan <= 0) return hipSuccess;
  if (g.rsb != 0 && g.rsb != (size_t)g.nl) return hipErrorInvalidValue;  // digit recode reads rows nl apart
  if (m.pad < MF_PAD_MIN || m.slices != m.S + 2 * m.pad || (size_t)m.slices * m.NT * 16 > 0x7fffffffu)
    return hipErrorInvalidValue;  // digit panels: padding and 32-bit buffer offsets
  // digits of the panel: b from the multiplier array, u from the panel buffer
  hipError_t e = launch_recode(g.Bop, g.ldb, g.npan, m.NT, m.NT, g.nl, m.pad, m.bdig, stream);
  if (e != hipSuccess) return e;
  e = launch_recode(g.Uop, g.ldu, g.npan, m.NT, m.u_rows, g.nl, m.pad, m.udig, stream);
  if (e != hipSuccess) return e;
  const int nt = m.NT / 32;
  int C_lo, nrow, ncol, ntiles;
  if (g.tri) {
    C_lo = g.c_lo / 32;
    nrow = ncol = nt - C_lo;
    ntiles = ncol * (ncol + 1) / 2;
  } else {
    C_lo = g.r_lo / 32;  // first tile row of the rectangular target
    nrow = nt - C_lo;
    ncol = g.ntc;
    ntiles = nrow * ncol;
  }
  RangeTab rt = make_ranges(g.nl, m.S, ntiles, m.max_ranges, m.carry_tiles);
  // one carry slot of 1024 entries per work item
  if (rt.n > m.max_ranges || (size_t)ntiles * rt.n > m.carry_tiles) return hipErrorInvalidValue;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (m.timing) {
    (void)hipEventCreate(&ev0);
    (void)hipEventCreate(&ev1);
    (void)hipEventRecord(ev0, stream);
  }
  const long items = (long)ntiles * rt.n;
  const int per_xcd = (int)((items + 7) / 8);
  hipLaunchKernelGGL(k_upd_mfma, dim3(8 * per_xcd), dim3(64), 0, stream, m, rt, C_lo, ntiles, per_xcd);
  e = hipGetLastError();
  if (m.timing) {
    (void)hipEventRecord(ev1, stream);
    (void)hipEventSynchronize(ev1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ev0, ev1);
    m.timing->ms[6] += ms;
    m.timing->launches[1] += 1;
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
  }
  if (e != hipSuccess) return e;
  if (rt.n > 1) {
    hipLaunchKernelGGL(k_carry_fix, dim3(nrow, ncol), dim3(1024), 0, stream, m, rt, C_lo);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_kara_gemm(const KaraArgs& k, const RangeTab& rt, int C_lo, int ntiles, int per_xcd,
                            hipStream_t stream) {
  hipLaunchKernelGGL(k_upd_kara, dim3(8 * per_xcd), dim3(64), 0, stream, k, rt, C_lo, ntiles, per_xcd);
  return hipGetLastError();
}

hipError_t launch_recode_batch(const RecodeArgs* tab, int count, int rows_limbs_max, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const size_t threads = (size_t)rows_limbs_max * 16;
  hipLaunchKernelGGL(k_recode_b, dim3((unsigned)((threads + 255) / 256), count), dim3(256), 0, stream, tab);
  return hipGetLastError();
}

hipError_t launch_upd_mfma_batch(const MfmaEntry* tab, const int4* items, int per_xcd, unsigned* heads,
                                 hipStream_t stream) {
  if (per_xcd <= 0) return hipSuccess;
  hipError_t e = launch_fill(heads, 8, 0u, stream);
  if (e != hipSuccess) return e;
  // one wave per SIMD of each XCD (32 CUs x 4), no more than the queue holds
  const int waves = per_xcd < 128 ? per_xcd : 128;
  hipLaunchKernelGGL(k_upd_mfma_b, dim3(8 * waves), dim3(64), 0, stream, tab, items, per_xcd, heads);
  return hipGetLastError();
}

hipError_t launch_carry_fix_batch(const MfmaEntry* tab, int count, int nrow_max, int ncol_max, hipStream_t stream) {
  if (count <= 0 || nrow_max <= 0 || ncol_max <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_carry_fix_b, dim3(nrow_max, ncol_max, count), dim3(1024), 0, stream, tab);
  return hipGetLastError();
}

hipError_t launch_mfma_probe(int* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, stream, out);
  return hipGetLastError();
}

}  // namespace hl
