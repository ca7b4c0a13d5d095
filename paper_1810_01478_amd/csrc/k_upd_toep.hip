// Exact update A[r][c] <- A[r][c] - sum_{i in panel} b_ri u_ci as int8 MFMA
// GEMMs in Toeplitz form, for targets with few columns: the updates inside a
// panel of the LDL^T (rank 1), the triangular solve with k right-hand sides and
// the adjoint's back substitution (Algorithm 1 and the solves of Section 3).
//
// Digits.  As in the slice form, each P-bit two's complement factor is recoded
// into S = P/8 balanced base-256 digits, and entry (r, c) receives
//   sum_t 256^t out_t(r, c),  out_t(r, c) = sum_i sum_j beta_{r,i,j} upsilon_{c,i,t-j}.
// The slice form takes K over the 16 panel columns, which wastes most of each
// MFMA when the panel has one column or the target has fewer than 32.  Here, for
// one column c and factor column i, 32 rows x 32 consecutive output digits
// t0..t0+31 x 32 consecutive digits j0..j0+31 is one GEMM
//   out[t][r] += sum_j U[t][j] B[j][r],  U[t][j] = upsilon_{c,i,t-j} (Toeplitz),
// B[j][r] = beta_{r,i,j}.  v_mfma_i32_32x32x32_i8 takes the Toeplitz operand as
// its first (M = output digits) and the b digits as its second (N = rows); the
// output digit of MFMA row m is chosen so that each lane ends up holding 16
// consecutive digits (4 limbs) of one entry.
//
// Kernel.  One wave owns 32 rows x one column x TP_DIGITS = 512 output digits
// (16 accumulators of 32 digits).  Step s multiplies digits j0 = jb + 32 s: the
// accumulator of output block q needs the Toeplitz window for t0 + 32 q - j0,
// which is the window accumulator q - 1 used at step s - 1, so a ring of 16
// windows turns by one per step: each step loads one window (two aligned
// 16-byte chunks, shifted into place with v_alignbyte by the lane's offset) and
// one 16-byte run of b digits, and issues 16 MFMAs.  The u digits are stored
// reversed so that a window is a forward run of bytes.  Digits outside [0, S)
// are zero padding.
//
// Recombination.  Each lane folds its 16 digit sums of a 4-limb chunk into
// A - sum_t 256^t out_t (exact, 128 bits plus a small carry); the carries then
// run through the 32 chunks of the item in order, alternating between the two
// lane halves.  The carry out of the item's limb range is stored and added by
// k_toep_carry, so the ranges of one entry run in parallel.
#include "hl_kernels.hpp"

namespace hl {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int TP_Q = TP_DIGITS / 32;  // accumulators (output blocks of 32 digits)
constexpr int TP_PF = 4;              // operands are loaded this many steps ahead
constexpr int TP_ROT = TP_Q;          // steps per unrolled rotation of the window ring
static_assert(TP_Q == 16, "the lane layout below assumes 16 blocks of 32 digits");
static_assert(TP_ROT % TP_PF == 0, "the load rings must turn a whole number of times per rotation");
// padding: with n_s steps rounded up to whole rotations, windows are loaded for
// d in [-(TP_Q-1), n_s + TP_ROT - 1 + TP_PF] and b runs for steps up to
// n_s + TP_ROT - 2 + TP_PF (see toep_item)
static_assert(TP_PADB >= 32 * (TP_ROT - 2 + TP_PF) + 64, "b padding");
static_assert(TP_PADU_LO >= 32 * TP_Q + 32, "u padding below");
static_assert(TP_PADU_HI >= TP_DIGITS + 32 * (TP_ROT + TP_PF) + 48, "u padding above");

__device__ __forceinline__ v4i tp_ld16(const int8_t* p) { return *(const v4i*)p; }

// 16 bytes at byte offset 4 aw + ab of the 32 bytes (lo, hi): two rounds of
// selects by the bits of aw, then byte funnel shifts
__device__ __forceinline__ v4i tp_window(v4i lo, v4i hi, int aw, int ab) {
  const bool s2 = (aw & 2) != 0, s1 = (aw & 1) != 0;
  const u32 f0 = s2 ? (u32)lo.z : (u32)lo.x, f1 = s2 ? (u32)lo.w : (u32)lo.y;
  const u32 f2 = s2 ? (u32)hi.x : (u32)lo.z, f3 = s2 ? (u32)hi.y : (u32)lo.w;
  const u32 f4 = s2 ? (u32)hi.z : (u32)hi.x, f5 = s2 ? (u32)hi.w : (u32)hi.y;
  const u32 e0 = s1 ? f1 : f0, e1 = s1 ? f2 : f1, e2 = s1 ? f3 : f2, e3 = s1 ? f4 : f3, e4 = s1 ? f5 : f4;
  v4i o;
  o.x = (int)__builtin_amdgcn_alignbyte(e1, e0, (u32)ab);
  o.y = (int)__builtin_amdgcn_alignbyte(e2, e1, (u32)ab);
  o.z = (int)__builtin_amdgcn_alignbyte(e3, e2, (u32)ab);
  o.w = (int)__builtin_amdgcn_alignbyte(e4, e3, (u32)ab);
  return o;
}

// Output digit (within a block of 32) of row m of the MFMA result: chosen so
// that lane l, register v of the result holds digit 16 (l >> 5) + v.
__device__ __forceinline__ int tp_digit_of_row(int m) { return 16 * ((m >> 2) & 1) + 4 * (m >> 3) + (m & 3); }

// limb Lq of target entry (r, c)
__device__ __forceinline__ u32* tp_entry(const ToepArgs& a, int r, int c, int Lq) {
  const UpdArgs& g = a.g;
  if (a.plain) return g.A + (size_t)r * a.ldr + (size_t)c * a.ldc + Lq;
  const size_t tix = g.tri ? tri_tile_index(r >> 5, c >> 5) : (size_t)(r >> 5) * g.ntc + (c >> 5);
  return g.A + tix * tile_words(g.nw) + in_tile(r, c, Lq);
}

// one accumulator register, read by itself (taking an element of the vector
// otherwise copies the whole vector out of the accumulation registers)
__device__ __forceinline__ int tp_acc(int v) {
  int o;
  asm("v_accvgpr_read_b32 %0, %1" : "=v"(o) : "a"(v));
  return o;
}
// acc * m + d as one 32 x 32 -> 64-bit signed multiply-add (m opaque, so that
// a power of two does not become 64-bit shifts)
__device__ __forceinline__ i64 tp_mad(int acc, int m, i64 d) { return (i64)acc * (i64)m + d; }
__device__ __forceinline__ int tp_opaque(int v) {
  asm volatile("" : "+s"(v));
  return v;
}

// One work item: rows 32 RB .. 32 RB + 31, column c_lo + cc, output digits
// [512 rg, 512 rg + 512); the carry out of the range goes to cb[0..31].
__device__ __forceinline__ void toep_item(const ToepArgs& a, int rg, int RB, int cc, long long* cb) {
  const UpdArgs& g = a.g;
  if (has_error(g.st)) return;
  const int l = lane_id(), h = l >> 5, n = l & 31;
  const int Sb = a.Sb, Su = a.Su;
  const int BS = tp_bstride(Sb), US = tp_ustride(Su);
  const int t0 = TP_DIGITS * rg;
  v16i acc[TP_Q];
#pragma unroll
  for (int q = 0; q < TP_Q; ++q) acc[q] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  // digit j of b pairs with digit t - j of u: j in [t - (Su-1), t] and [0, Sb)
  int jlo = t0 - (Su - 1);
  if (jlo < 0) jlo = 0;
  int jhi = t0 + TP_DIGITS - 1;
  if (jhi > Sb - 1) jhi = Sb - 1;
  if (jlo <= jhi) {
    const int jb = jlo & ~31;
    const int n_s = (jhi - jb) / 32 + 1;
    const int nrot = (n_s + TP_ROT - 1) / TP_ROT;
    // Window d (accumulator q at step s uses d = s - q) of this lane (A row m = n,
    // K half h) holds upsilon_{T - x}, x = 0..15, T = t0 + t(m) - jb - 16 h - 32 d,
    // i.e. reversed digits Su-1-T .. Su-1-T+15: byte offset wb + 32 d of the padded row.
    const int wb = TP_PADU_LO + Su - 1 - t0 - tp_digit_of_row(n) + 16 * h + jb;
    const int aoff = wb & 15, aw = aoff >> 2, ab = aoff & 3;
    for (int p = 0; p < g.npan; ++p) {
      const int8_t* ur = a.ud + ((size_t)p * a.ncols + cc) * US + (wb & ~15);
      const int8_t* br = a.bd + ((size_t)p * a.NT + (size_t)RB * 32 + n) * BS + jb + 16 * h;
      // ring: slot d mod 16 holds window d; step s first multiplies accumulator
      // 15 (window s - 15), then shifts window s + 1 into that slot, so each
      // window is ready a step before its first use
      v4i win[TP_Q];
#pragma unroll
      for (int d = -(TP_Q - 1); d <= 0; ++d)
        win[(d + TP_Q) % TP_Q] = tp_window(tp_ld16(ur + 32 * d), tp_ld16(ur + 32 * d + 16), aw, ab);
      v4i rlo[TP_PF], rhi[TP_PF], bq[TP_PF];
#pragma unroll
      for (int d = 1; d <= TP_PF; ++d) {
        rlo[d % TP_PF] = tp_ld16(ur + 32 * d);
        rhi[d % TP_PF] = tp_ld16(ur + 32 * d + 16);
      }
#pragma unroll
      for (int s = 0; s < TP_PF; ++s) bq[s] = tp_ld16(br + 32 * s);
      const int8_t* un = ur + 32 * (TP_PF + 1);  // raw window s + 1 + TP_PF, loaded at step s
      const int8_t* bn = br + 32 * TP_PF;        // b digits of step s + TP_PF, loaded at step s
      for (int rot = 0; rot < nrot; ++rot) {
        const int s_end = n_s - rot * TP_ROT;  // steps of this rotation that multiply
#pragma unroll
        for (int st = 0; st < TP_ROT; ++st) {
          const v4i bv = bq[st % TP_PF];
          const bool run = st < s_end;
          if (run)
            acc[TP_Q - 1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(win[(st + 1) % TP_Q], bv, acc[TP_Q - 1], 0, 0, 0);
          win[(st + 1) % TP_Q] = tp_window(rlo[(st + 1) % TP_PF], rhi[(st + 1) % TP_PF], aw, ab);
          rlo[(st + 1) % TP_PF] = tp_ld16(un);
          rhi[(st + 1) % TP_PF] = tp_ld16(un + 16);
          bq[st % TP_PF] = tp_ld16(bn);
          un += 32;
          bn += 32;
          if (run) {
#pragma unroll
            for (int q = TP_Q - 2; q >= 0; --q)
              acc[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(win[(st - q + TP_Q) % TP_Q], bv, acc[q], 0, 0, 0);
          }
        }
      }
    }
  }
  // entry (r, c) of this lane; lane half h holds chunks (q, h): limbs L0 + 8 q ..
  // L0 + 8 q + 3
  const int r = RB * 32 + n, c = g.c_lo + cc;
  const bool live = r >= g.r_lo && r < g.r_hi && c < g.c_hi && (!g.tri || r >= c);
  const int L0 = t0 / 4 + 4 * h;
  uint4 x[TP_Q];
#pragma unroll
  for (int q = 0; q < TP_Q; ++q) {
    const int Lq = L0 + 8 * q;
    x[q] = (live && Lq < g.nw && a.add != 2) ? *(const uint4*)tp_entry(a, r, c, Lq) : make_uint4(0, 0, 0, 0);
  }
  // x -/+ sum_v 256^v out_v per chunk, 32 bits at a time: limb k takes the
  // digit sums 4k .. 4k + 3 (one 32 x 32 -> 64-bit multiply-add each, the
  // multipliers +-2^(8m) opaque) and the carry of limb k - 1; the chunk's carry
  // (below 2^25 in magnitude) goes to zc
  const int sg = a.add ? 1 : -1;
  const int m0 = tp_opaque(sg), m8 = tp_opaque(sg << 8), m16 = tp_opaque(sg << 16), m24 = tp_opaque(sg * (1 << 24));
  const int one = tp_opaque(1);
  int zc[TP_Q];
#pragma unroll
  for (int q = 0; q < TP_Q; ++q) {
    const u32 xa[4] = {x[q].x, x[q].y, x[q].z, x[q].w};
    i64 t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      i64 y = (i64)xa[k];
      y = tp_mad(tp_acc(acc[q][4 * k]), m0, y);
      y = tp_mad(tp_acc(acc[q][4 * k + 1]), m8, y);
      y = tp_mad(tp_acc(acc[q][4 * k + 2]), m16, y);
      t[k] = tp_mad(tp_acc(acc[q][4 * k + 3]), m24, y);
    }
#pragma unroll
    for (int k = 1; k < 4; ++k) t[k] = tp_mad((int)(t[k - 1] >> 32), one, t[k]);
    x[q] = make_uint4((u32)t[0], (u32)t[1], (u32)t[2], (u32)t[3]);
    zc[q] = (int)(t[3] >> 32);
  }
  // carries through the chunks in limb order: (0,0), (0,1), (1,0), ...
  i64 carry = 0;
#pragma unroll
  for (int k = 0; k < 2 * TP_Q; ++k) {
    const int q = k >> 1, half = k & 1;
    i64 cout = 0;
    if (h == half) {
      const unsigned __int128 U = ((unsigned __int128)(((u64)x[q].w << 32) | x[q].z) << 64) |
                                  (((u64)x[q].y << 32) | x[q].x);
      const unsigned __int128 V = U + (unsigned __int128)(__int128)carry;
      const int delta = carry >= 0 ? (V < U ? 1 : 0) : (V > U ? -1 : 0);
      const u64 lo = (u64)V, hi = (u64)(V >> 64);
      x[q] = make_uint4((u32)lo, (u32)(lo >> 32), (u32)hi, (u32)(hi >> 32));
      cout = (i64)zc[q] + delta;
    }
    carry = __shfl(cout, half * 32 + n, WAVE);
  }
#pragma unroll
  for (int q = 0; q < TP_Q; ++q) {
    const int Lq = L0 + 8 * q;
    if (live && Lq < g.nw) *(uint4*)tp_entry(a, r, c, Lq) = x[q];
  }
  if (h == 0) cb[n] = live ? carry : 0;
}

// Item of block b.  Workgroups go to the 8 XCDs in turn (block b to XCD
// b mod 8); the G = ncols items of one range and row block (consecutive
// columns) are given to one XCD in consecutive slots, so that the 16-byte
// pieces their epilogues read and write of each 128-byte line of the target
// tiles (8 columns of one row) meet in that XCD's L2.  Bijective: whole rounds
// of 8 groups are permuted, the remainder keeps its order.
__device__ __forceinline__ int toep_item_of_block(int b, int nitems, int G) {
  const int full = nitems / (8 * G) * (8 * G);
  if (G <= 1 || b >= full) return b;
  const int x = b & 7, t = b >> 3;
  return ((t / G) * 8 + x) * G + t % G;
}

// Work items (range, row block, column) in range-major order, the ranges with
// the most steps first; block b takes item b, so the workgroups dealt to the
// 8 XCDs in turn give every XCD the same mix of long and short items, and the
// short ones fill in at the end.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_upd_toep(ToepArgs a) {
  const int per_rg = a.nrb * a.ncols;
  const int item = toep_item_of_block((int)blockIdx.x, a.nrg * per_rg, a.ncols);
  if (item >= a.nrg * per_rg) return;
  const int k = item / per_rg, rem = item - k * per_rg;
  const int rg = a.rg_order[k];  // longest ranges are dealt first
  const int rb = rem / a.ncols, cc = rem - rb * a.ncols;
  toep_item(a, rg, a.RB_lo + rb, cc, a.carry + ((size_t)rg * per_rg + rem) * 32);
}

// batch: blockIdx.y is the record (npan <= 0 skips it)
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_upd_toep_b(const ToepArgs* __restrict__ tab) {
  const ToepArgs& a = tab[blockIdx.y];
  if (a.g.npan <= 0) return;
  const int item = blockIdx.x;
  const int per_rg = a.nrb * a.ncols;
  if (item >= a.nrg * per_rg) return;
  const int k = item / per_rg, rem = item - k * per_rg;
  const int rg = a.rg_order[k];
  const int rb = rem / a.ncols, cc = rem - rb * a.ncols;
  toep_item(a, rg, a.RB_lo + rb, cc, a.carry + ((size_t)rg * per_rg + rem) * 32);
}

// Add the carry of range w at limb 128 (w + 1) of every entry, w = 0 .. nrg-2
// (one thread per entry of the target).  The ranges' carries go in as 64-bit
// adds on their own limb pairs, eight ranges at a time with all loads issued
// together; an add that carries out of its pair is finished afterwards by
// rippling +-1 upwards (rare).  Additions commute, so the order is free.
__device__ __forceinline__ void toep_carry_body(const ToepArgs& a, int e) {
  const UpdArgs& g = a.g;
  if (e >= a.nrb * 32 * a.ncols) return;
  if (has_error(g.st)) return;
  const int rr = e / a.ncols, cc = e - rr * a.ncols;
  const int rb = rr >> 5, n = rr & 31;
  const int r = (a.RB_lo + rb) * 32 + n, c = g.c_lo + cc;
  if (!(r >= g.r_lo && r < g.r_hi && c < g.c_hi && (!g.tri || r >= c))) return;
  const int nw = g.nw;
  const size_t per_rg = (size_t)a.nrb * a.ncols;
  const long long* cbase = a.carry + ((size_t)rb * a.ncols + cc) * 32 + n;
  constexpr int G = 8;
  for (int w0 = 0; w0 + 1 < a.nrg; w0 += G) {
    i64 cv[G];
    u64 xv[G];
    u32* pp[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int w = w0 + k, li = (TP_DIGITS / 4) * (w + 1);
      const bool ok = w + 1 < a.nrg && li < nw;
      cv[k] = ok ? cbase[(size_t)w * per_rg * 32] : 0;
      pp[k] = tp_entry(a, r, c, ok ? li : 0);
      xv[k] = ok ? (((u64)pp[k][1] << 32) | pp[k][0]) : 0;
    }
    int dir[G];  // what the pair's add passes to the limbs above: 0, +1 or -1
#pragma unroll
    for (int k = 0; k < G; ++k) {
      dir[k] = 0;
      if (cv[k] == 0) continue;
      const u64 s2 = xv[k] + (u64)cv[k];
      pp[k][0] = (u32)s2;
      pp[k][1] = (u32)(s2 >> 32);
      // the sign-extended add of cv: +1 when the unsigned add wrapped, and the
      // extension of a negative cv contributes -1 above the pair
      dir[k] = (s2 < xv[k] ? 1 : 0) + (cv[k] < 0 ? -1 : 0);
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      if (dir[k] == 0) continue;
      const u64 add = dir[k] > 0 ? 1ull : ~0ull;
      for (int li = (TP_DIGITS / 4) * (w0 + k + 1) + 2; li < nw; li += 2) {
        u32* p = tp_entry(a, r, c, li);
        const u64 x = ((u64)p[1] << 32) | p[0];
        const u64 y = x + add;
        p[0] = (u32)y;
        p[1] = (u32)(y >> 32);
        if (dir[k] > 0 ? (y != 0) : (x != 0)) break;  // the carry or borrow stops here
      }
    }
  }
}

// ---------------------------------------------------------------------------

__global__ void k_toep_carry(ToepArgs a) { toep_carry_body(a, blockIdx.x * blockDim.x + threadIdx.x); }

__global__ void k_toep_carry_b(const ToepArgs* __restrict__ tab) {
  const ToepArgs& a = tab[blockIdx.y];
  if (a.g.npan > 0 && a.nrg > 1) toep_carry_body(a, blockIdx.x * blockDim.x + threadIdx.x);
}

// b digits, forward: bd[p][row][j], rows 32 RB_lo .. 32 (RB_lo + nrb) - 1
// (rows outside [r_lo, r_hi) read as zero), zero for j >= Sb.
__device__ __forceinline__ void toep_recode_b_body(const ToepArgs& a, size_t gid) {
  const UpdArgs& g = a.g;
  const int BS4 = tp_bstride(a.Sb) / 4;
  const size_t rows = (size_t)a.nrb * 32;
  if (gid >= (size_t)g.npan * rows * BS4) return;
  const int w = (int)(gid % BS4);
  const size_t pr = gid / BS4;
  const int p = (int)(pr / rows);
  const int row = a.RB_lo * 32 + (int)(pr % rows);
  u32 v = 0;
  if (4 * w < a.Sb && row >= g.r_lo && row < g.r_hi) {
    const size_t rsb = g.rsb ? g.rsb : (size_t)a.nlb;
    v = balanced_digits4(g.Bop + (size_t)p * g.ldb + (size_t)row * rsb, a.nlb, w);
  }
  u32* dst = (u32*)(a.bd + ((size_t)p * a.NT + row) * tp_bstride(a.Sb));
  dst[w] = v;
}

// u digits, reversed: ud[p][cc][TP_PADU_LO + y] = digit Su-1-y of u_(c_lo+cc), zero padded
__device__ __forceinline__ void toep_recode_u_body(const ToepArgs& a, size_t gid) {
  const UpdArgs& g = a.g;
  const int US4 = tp_ustride(a.Su) / 4;
  if (gid >= (size_t)g.npan * a.ncols * US4) return;
  const int w = (int)(gid % US4);
  const size_t pc = gid / US4;
  const int p = (int)(pc / a.ncols), cc = (int)(pc % a.ncols);
  const int y = 4 * w - TP_PADU_LO;
  u32 v = 0;
  if (y >= 0 && y < a.Su) {
    // bytes y .. y+3 are digits Su-1-y .. Su-4-y: limb nlu-1-y/4, reversed
    const int c = g.c_lo + cc;
    v = __builtin_bswap32(balanced_digits4(g.Uop + (size_t)p * g.ldu + (size_t)c * a.ucs, a.nlu, a.nlu - 1 - y / 4));
  }
  u32* dst = (u32*)(a.ud + ((size_t)p * a.ncols + cc) * tp_ustride(a.Su));
  dst[w] = v;
}

__global__ void k_toep_recode_b(ToepArgs a) { toep_recode_b_body(a, (size_t)blockIdx.x * blockDim.x + threadIdx.x); }
__global__ void k_toep_recode_u(ToepArgs a) { toep_recode_u_body(a, (size_t)blockIdx.x * blockDim.x + threadIdx.x); }
__global__ void k_toep_recode_b_b(const ToepArgs* __restrict__ tab) {
  const ToepArgs& a = tab[blockIdx.y];
  if (a.g.npan > 0) toep_recode_b_body(a, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void k_toep_recode_u_b(const ToepArgs* __restrict__ tab) {
  const ToepArgs& a = tab[blockIdx.y];
  if (a.g.npan > 0) toep_recode_u_body(a, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Host: fill in the derived fields of a (launch extents, range order) and check
// the capacities.  *empty when there is nothing to update.
hipError_t toep_prepare(ToepArgs& a, bool* empty) {
  const UpdArgs& g = a.g;
  *empty = g.r_hi <= g.r_lo || g.c_hi <= g.c_lo || g.npan <= 0;
  if (*empty) return hipSuccess;
  if (a.nlb <= 0) a.nlb = g.nl;
  if (a.nlu <= 0) a.nlu = g.nl;
  if (a.ucs == 0) a.ucs = (size_t)a.nlu;
  a.Sb = 4 * a.nlb;
  a.Su = 4 * a.nlu;
  // digit sums stay below 2^31: npan x min(Sb, Su) x 2^14
  const int smin = a.Sb < a.Su ? a.Sb : a.Su;
  if (g.npan > 16 || (long)g.npan * smin > 131071 || g.nw < 1 || (g.nw & 3)) return hipErrorInvalidValue;
  if (!a.plain && g.nw != 2 * g.nl) return hipErrorInvalidValue;
  if (a.plain && ((a.ldr & 3) || (a.ldc & 3) || ((uintptr_t)g.A & 15))) return hipErrorInvalidValue;
  a.RB_lo = g.r_lo / 32;
  a.nrb = (g.r_hi - 1) / 32 + 1 - a.RB_lo;
  a.ncols = g.c_hi - g.c_lo;
  a.nrg = tp_ranges(g.nw);
  if (a.nrg > TP_MAX_RANGES) return hipErrorInvalidValue;
  {
    // steps of each output range (as toep_item counts them), longest first
    int steps[TP_MAX_RANGES];
    for (int rg = 0; rg < a.nrg; ++rg) {
      const int t0 = TP_DIGITS * rg;
      const int jlo = t0 - (a.Su - 1) > 0 ? t0 - (a.Su - 1) : 0;
      const int jhi = t0 + TP_DIGITS - 1 < a.Sb - 1 ? t0 + TP_DIGITS - 1 : a.Sb - 1;
      steps[rg] = jlo <= jhi ? (jhi - (jlo & ~31)) / 32 + 1 : 0;
      a.rg_order[rg] = (unsigned char)rg;
    }
    for (int i = 1; i < a.nrg; ++i)  // stable insertion sort, descending
      for (int j = i; j > 0 && steps[a.rg_order[j]] > steps[a.rg_order[j - 1]]; --j) {
        const unsigned char t = a.rg_order[j];
        a.rg_order[j] = a.rg_order[j - 1];
        a.rg_order[j - 1] = t;
      }
  }
  if ((a.RB_lo + a.nrb) * 32 > a.NT) return hipErrorInvalidValue;
  const size_t rows = (size_t)a.nrb * 32;
  const size_t bneed = ((size_t)(g.npan - 1) * a.NT + (size_t)(a.RB_lo + a.nrb) * 32) * tp_bstride(a.Sb);
  const size_t uneed = (size_t)g.npan * a.ncols * tp_ustride(a.Su);
  const long items = (long)a.nrg * a.nrb * a.ncols;
  if (bneed > a.bd_bytes || uneed > a.ud_bytes || (size_t)items * 32 > a.carry_words) return hipErrorInvalidValue;
  (void)rows;
  return hipSuccess;
}

// launch extents of a prepared record: recode threads (b, u), work items, entries
void toep_extents(const ToepArgs& a, size_t* nb, size_t* nu, size_t* items, size_t* entries) {
  const size_t rows = (size_t)a.nrb * 32;
  *nb = (size_t)a.g.npan * rows * (tp_bstride(a.Sb) / 4);
  *nu = (size_t)a.g.npan * a.ncols * (tp_ustride(a.Su) / 4);
  *items = (size_t)a.nrg * a.nrb * a.ncols;
  *entries = rows * a.ncols;
}

hipError_t launch_upd_toep(const ToepArgs& a0, hipStream_t stream) {
  ToepArgs a = a0;
  bool empty = false;
  hipError_t e0 = toep_prepare(a, &empty);
  if (e0 != hipSuccess || empty) return e0;
  const UpdArgs& g = a.g;
  const size_t rows = (size_t)a.nrb * 32;
  const long items = (long)a.nrg * a.nrb * a.ncols;
  {
    const size_t n = (size_t)g.npan * rows * (tp_bstride(a.Sb) / 4);
    hipLaunchKernelGGL(k_toep_recode_b, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    const size_t n = (size_t)g.npan * a.ncols * (tp_ustride(a.Su) / 4);
    hipLaunchKernelGGL(k_toep_recode_u, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_upd_toep, dim3((unsigned)items), dim3(64), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.nrg < 2) return e;
  const size_t ne = rows * a.ncols;
  hipLaunchKernelGGL(k_toep_carry, dim3((unsigned)((ne + 63) / 64)), dim3(64), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_upd_toep_batch(const ToepArgs* tab, int count, size_t nb_max, size_t nu_max, size_t items_max,
                                size_t entries_max, int nrg_max, hipStream_t stream) {
  if (count <= 0 || items_max == 0) return hipSuccess;
  hipLaunchKernelGGL(k_toep_recode_b_b, dim3((unsigned)((nb_max + 255) / 256), count), dim3(256), 0, stream, tab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_toep_recode_u_b, dim3((unsigned)((nu_max + 255) / 256), count), dim3(256), 0, stream, tab);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_upd_toep_b, dim3((unsigned)items_max, count), dim3(64), 0, stream, tab);
  e = hipGetLastError();
  if (e != hipSuccess || nrg_max < 2) return e;
  hipLaunchKernelGGL(k_toep_carry_b, dim3((unsigned)((entries_max + 255) / 256), count), dim3(256), 0, stream, tab);
  return hipGetLastError();
}

}  // namespace hl
