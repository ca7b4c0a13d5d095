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
#include <utility>

#include "hl_kernels.hpp"

namespace hl {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int MF_T = 16;             // output digits per accumulation block
constexpr int MF_LPB = MF_T / 4;     // limbs per block (one 16-byte slab of an entry)
constexpr int MF_PF = 8;             // operands are loaded this many steps ahead
constexpr int MF_WIN = MF_T + 2 * MF_PF;  // B window: MF_T slices in use, the rest in flight
constexpr int MF_ROT = MF_WIN / 2;   // steps per rotation of the window (a multiple of MF_PF)
static_assert(MF_ROT % MF_PF == 0, "the A ring must turn a whole number of times per rotation");
// zero slices needed at each end of the digit panels: the loads run MF_PF steps
// (2 MF_PF slices) ahead and the steps are rounded up to whole rotations
constexpr int MF_PAD_MIN = 2 * (MF_ROT + MF_PF) + 14;

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
constexpr int kRawBufferWord3 = 0x00020000;  // gfx9 buffer descriptor word 3 (32-bit data format)

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
template <bool STORE>
__device__ __forceinline__ void mfma_tile_t(const UpdArgs& g, const int8_t* bdig, const int8_t* udig, int slices,
                                            int S, int pad, int NT, int R, int C, int tb0, int tb1, long long* cb,
                                            u32* Out) {
  if (has_error(g.st)) return;
  __shared__ i64 carry_s[16 * WAVE];  // carry of each of the lane's 16 entries
  const int l = lane_id(), h = l >> 5, mm = l & 31;
  const int sst = NT * 16;  // bytes per digit slice
  // A operand (b digits of tile rows), B operand (u digits of tile columns),
  // read through buffer descriptors: a 32-bit lane offset plus a wave-uniform
  // slice offset stepped in scalar registers, so no load in flight holds a
  // per-lane 64-bit address
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<int8_t*>(bdig), 0, slices * sst, kRawBufferWord3);
  const __amdgpu_buffer_rsrc_t ru =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<int8_t*>(udig), 0, slices * sst, kRawBufferWord3);
  const int aoff = h * sst + R * 512 + mm * 16;
  const int uoff = (1 - h) * sst + C * 512 + mm * 16;
  unsigned live = 0;  // entries of the trailing matrix proper (r >= c, inside the target)
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    carry_s[v * WAVE + l] = 0;
    const int r = R * 32 + mf_row(l, v), c = C * 32 + mf_col(l);
    if ((!g.tri || r >= c) && r >= g.r_lo && r < g.r_hi && c >= g.c_lo && c < g.c_hi) live |= 1u << v;
  }
  for (int tb = tb0; tb < tb1; ++tb) {
    const int t0 = MF_T * tb;
    v16i acc[MF_T];
#pragma unroll
    for (int q = 0; q < MF_T; ++q) acc[q] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    int jlo = t0 - (S - 1);
    if (jlo < 0) jlo = 0;
    jlo &= ~1;
    int jhi = t0 + MF_T - 1;
    if (jhi > S - 1) jhi = S - 1;
    // steps of two digits, padded to whole rotations of the register window;
    // the extra steps pair A digits with zero B padding (or the reverse) and
    // add nothing
    const int nsteps = (jhi - jlo) / 2 + 1;
    const int nrot = (nsteps + MF_ROT - 1) / MF_ROT;
    // Window slot (y mod MF_WIN) holds the slice at offset t0 - jlo + y; step s
    // multiplies y = q - 2s for q = 0..MF_T-1 and loads y = -2 MF_PF - 2s,
    // -2 MF_PF + 1 - 2s for step s + MF_PF.  A digits are likewise loaded
    // MF_PF steps ahead into a ring.
    const int ub = (pad - 1 + t0 - jlo) * sst;
    v4i w[MF_WIN];
#pragma unroll
    for (int y = 0; y < MF_T; ++y) w[y] = bld16(ru, uoff, ub + y * sst);
#pragma unroll
    for (int y = -2 * (MF_PF - 1); y < 0; ++y) w[MF_WIN + y] = bld16(ru, uoff, ub + y * sst);
    int ap = (pad + jlo) * sst;
    v4i an[MF_PF];
#pragma unroll
    for (int q = 0; q < MF_PF; ++q) an[q] = bld16(rb, aoff, ap + 2 * q * sst);
    ap += 2 * MF_PF * sst;
    int un = ub - 2 * MF_PF * sst;
    // Let the prologue's loads land here, once per block: the loop header then
    // only sees the loads in flight from the previous rotation, and its wait
    // keeps the MF_PF steps of prefetch instead of draining them every rotation.
    __builtin_amdgcn_s_waitcnt(kVmcntZero);
    for (int rot = 0; rot < nrot; ++rot) {
#pragma unroll
      for (int st = 0; st < MF_ROT; ++st) {
        const v4i a = an[st % MF_PF];
        an[st % MF_PF] = bld16(rb, aoff, ap);
        const int k0 = (MF_WIN * 4 - 2 * MF_PF - 2 * st) % MF_WIN;  // slot of y = -2 MF_PF - 2 st (even)
        w[k0] = bld16(ru, uoff, un);
        w[k0 + 1] = bld16(ru, uoff, un + sst);
#pragma unroll
        for (int q = 0; q < MF_T; ++q)
          acc[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, w[(q - 2 * st + MF_WIN * 4) % MF_WIN], acc[q], 0, 0, 0);
        ap += 2 * sst;
        un -= 2 * sst;
        __builtin_amdgcn_sched_group_barrier(0x020, 3, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, MF_T, 0);
      }
    }
    // fold the 16 digit sums of each entry into limbs 4 tb .. 4 tb + 3 (one slab)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      if (!((live >> v) & 1u)) continue;
      const int r = mf_row(l, v), c = mf_col(l);
      uint4* p = (uint4*)(Out + in_tile(r, c, MF_LPB * tb));
      i64 d[4] = {0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < MF_T; ++q) d[q >> 2] += (i64)acc[q][v] << (8 * (q & 3));
      __int128 X, Y;
      if (STORE) {
        X = (__int128)d[0] + ((__int128)d[1] << 32) + (__int128)carry_s[v * WAVE + l];
        Y = (__int128)d[2] + ((__int128)d[3] << 32) + (__int128)(i64)(X >> 64);
      } else {
        const uint4 x = *p;
        X = (__int128)(((u64)x.y << 32) | x.x) - (__int128)d[0] - ((__int128)d[1] << 32) +
            (__int128)carry_s[v * WAVE + l];
        Y = (__int128)(((u64)x.w << 32) | x.z) - (__int128)d[2] - ((__int128)d[3] << 32) + (__int128)(i64)(X >> 64);
      }
      const u64 lo = (u64)X, hi = (u64)Y;
      *p = make_uint4((u32)lo, (u32)(lo >> 32), (u32)hi, (u32)(hi >> 32));
      carry_s[v * WAVE + l] = (i64)(Y >> 64);
    }
  }
  // carries out of this range
#pragma unroll
  for (int v = 0; v < 16; ++v) cb[mf_row(l, v) * 32 + mf_col(l)] = carry_s[v * WAVE + l];
}

// the Schur update of tile (R, C) of the trailing matrix (see mfma_tile_t)
__device__ __forceinline__ void mfma_tile(const MfmaArgs& m, int R, int C, int tb0, int tb1, long long* cb) {
  const UpdArgs& g = m.g;
  const size_t tix = g.tri ? tri_tile_index(R, C) : (size_t)R * g.ntc + C;
  mfma_tile_t<false>(g, m.bdig, m.udig, m.slices, m.S, m.pad, m.NT, R, C, tb0, tb1, cb,
                     g.A + tix * tile_words(g.nw));
}

// tile (R, C) of work item lt of an entry's launch (see k_upd_mfma)
__device__ __forceinline__ void item_tile(const UpdArgs& g, int C_lo, int lt, int* R, int* C) {
  if (g.tri) {
    int r = (int)((sqrtf(8.0f * (float)lt + 1.0f) - 1.0f) * 0.5f);
    while (r > 0 && r * (r + 1) / 2 > lt) --r;
    while ((r + 1) * (r + 2) / 2 <= lt) ++r;
    *R = C_lo + r;
    *C = C_lo + (lt - r * (r + 1) / 2);
  } else {
    *R = C_lo + lt / g.ntc;
    *C = lt % g.ntc;
  }
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

// Batch of updates (one entry per instance) in one persistent launch.  Work
// items (entry, tile, range) sit in 8 queues, one per XCD, each largest first;
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
    mfma_tile(e.m, R, C, e.rt.tb[it.z], e.rt.tb[it.z + 1], e.m.carry + ((size_t)it.y * e.rt.n + it.z) * 1024);
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
  if (e.rt.n > 1) carry_fix_body(e.m, e.rt, e.C_lo, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Karatsuba form (see KaraArgs).
//
// Digits of the halves: limb q of a factor holds its balanced digits 4q..4q+3;
// those below h = 4 hq go to the lo panel, the others to the hi panel at digit
// 4q - h.  One thread per (limb, row, panel column), as recode_body.
__global__ void k_recode_kara(const u32* __restrict__ src, size_t lds, int npan, int NT, int nrows, int nl, int pad,
                              int hq, int8_t* __restrict__ lo, int8_t* __restrict__ hi) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int il = (int)(gid & 15);
  const size_t t = gid >> 4;
  const int row = (int)(t % NT), q = (int)(t / NT);
  if (q >= nl) return;
  const size_t rstride = (size_t)NT * 16;
  const int qq = q < hq ? q : q - hq;
  int8_t* d = (q < hq ? lo : hi) + (size_t)(pad + 4 * qq) * rstride + (size_t)row * 16 + il;
  u32 v = 0;
  if (il < npan && row < nrows) v = balanced_digits4(src + (size_t)il * lds + (size_t)row * nl, nl, q);
#pragma unroll
  for (int b = 0; b < 4; ++b) d[(size_t)b * rstride] = (int8_t)(v >> (8 * b));
}

// digits beyond S/2^l of level-l panel q (base-3 path, most significant digit
// first): lo children have none, hi children their parent's, mid children one more
__device__ __forceinline__ int kara_extra(int q, int l) {
  int e = 0, div = 1;
  for (int j = 1; j < l; ++j) div *= 3;
  for (int j = 0; j < l; ++j) {
    const int c = (q / div) % 3;
    e = c == 0 ? 0 : (c == 1 ? e : e + 1);
    div /= 3;
  }
  return e;
}

// floor((x + 128) / 256) for -512 <= x + 128: the balanced carry out of a
// digit position holding x
__device__ __forceinline__ int bal_carry(int x) { return (x + 640) / 256 - 2; }

// mid = lo + hi recoded into h + 1 balanced digits: sigma_j = lo_j + hi_j in
// [-256, 254], digit_j = sigma_j + c_j - 256 c_{j+1}, c_{j+1} = bal_carry(sigma_j
// + c_j) in {-1, 0, 1}, c_0 = 0; the top digit h is c_h.  One thread per (group
// of digits 4g..4g+3, row, panel column), g = 0..h/4; the carry into 4g is found
// by looking down to the nearest position whose carry out does not depend on
// the carry in, then carrying up from there.
__device__ __forceinline__ void kara_mid_body(const int8_t* __restrict__ lo, const int8_t* __restrict__ hi, int NT,
                                              int pad, int h, int8_t* __restrict__ mid) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int il = (int)(gid & 15);
  const size_t t = gid >> 4;
  const int row = (int)(t % NT), g = (int)(t / NT);
  if (g > h / 4) return;
  const size_t rs = (size_t)NT * 16, off = (size_t)row * 16 + il;
  auto sig = [&](int j) -> int {
    return j < h ? (int)lo[(size_t)(pad + j) * rs + off] + (int)hi[(size_t)(pad + j) * rs + off] : 0;
  };
  const int j0 = 4 * g;
  int js = j0 - 1;
  while (js >= 0) {
    const int sj = sig(js);
    if (bal_carry(sj - 1) == bal_carry(sj + 1)) break;
    --js;
  }
  int c = js >= 0 ? bal_carry(sig(js)) : 0;  // carry into js + 1
  for (int j = js + 1; j < j0; ++j) c = bal_carry(sig(j) + c);
  int8_t* d = mid + (size_t)(pad + j0) * rs + off;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int x = sig(j0 + b) + c;
    const int cn = bal_carry(x);
    d[(size_t)b * rs] = (int8_t)(x - 256 * cn);
    c = cn;
  }
}

__global__ void k_kara_mid(const int8_t* __restrict__ lo, const int8_t* __restrict__ hi, int NT, int pad, int h,
                           int8_t* __restrict__ mid) {
  kara_mid_body(lo, hi, NT, pad, h, mid);
}

// the mid children of every level-(l-1) panel (blockIdx.y, both sides): lo and
// hi child of n = S/2^(l-1) + extra digits, the hi child n - S/2^l of them
__global__ void k_kara_mid_lv(KaraArgs k, int l) {
  const int nq = kara_products(l - 1), y = blockIdx.y, side = y / nq, q = y - side * nq;
  const int s = k.m.S >> l;
  int8_t* lo = k.pan[l] + (size_t)(side * 3 * nq + 3 * q) * k.pan_stride[l];
  kara_mid_body(lo, lo + k.pan_stride[l], k.m.NT, k.m.pad, s + kara_extra(q, l - 1), lo + 2 * k.pan_stride[l]);
}

// Level l - 1 to level l: every panel q (blockIdx.y, both sides) has
// n = S/2^(l-1) + extra digits; slices [0, s) go to its lo child, [s, n) to its hi
// child (digit j - s), s = S/2^l.  One thread per 16 bytes of a slice.
__global__ void k_digit_split(KaraArgs k, int l) {
  const int nq = kara_products(l - 1), y = blockIdx.y, side = y / nq, q = y - side * nq;
  const int s = k.m.S >> l, n = 2 * s + kara_extra(q, l - 1), NT = k.m.NT, pad = k.m.pad;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = (int)(gid / NT), row = (int)(gid % NT);
  if (j >= n) return;
  const size_t rs = (size_t)NT * 16;
  const int8_t* src = k.pan[l - 1] + (size_t)y * k.pan_stride[l - 1];
  int8_t* lo = k.pan[l] + (size_t)(side * 3 * nq + 3 * q) * k.pan_stride[l];
  const uint4 v = *(const uint4*)(src + (size_t)(pad + j) * rs + (size_t)row * 16);
  int8_t* d = j < s ? lo + (size_t)(pad + j) * rs : lo + k.pan_stride[l] + (size_t)(pad + j - s) * rs;
  *(uint4*)(d + (size_t)row * 16) = v;
}

// The digit-sum GEMMs of the products: work items (range rg, product p, tile
// lt) in that order, dealt to the XCDs as in k_upd_mfma, so the waves of one
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
  mfma_tile_t<true>(g, leaf + (size_t)p * ls, leaf + (size_t)(np + p) * ls, k.kslices,
                    k.Sk, k.m.pad, k.m.NT, R, C, rt.tb[rg], rt.tb[rg + 1],
                    k.m.carry + (((size_t)p * ntiles + lt) * rt.n + rg) * 1024,
                    k.prod + ((size_t)p * k.prod_tiles + lt) * tile_words(k.nwp));
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
  static constexpr int NP = LV == 1 ? 3 : (LV == 2 ? 9 : 27);
  static constexpr int NT = LV == 1 ? 5 : (LV == 2 ? 25 : 125);
  KaTerm t[NT];
  int first[NP + 1];
  constexpr KaPoly() : t(), first() {
    int n = 0;
    for (int p = 0; p < NP; ++p) {
      first[p] = n;
      int pw[8] = {}, cf[8] = {}, m = 1;
      pw[0] = 0;
      cf[0] = 1;
      int div = NP / 3;
      for (int l = 1; l <= LV; ++l) {
        const int c = (p / div) % 3;
        div = div / 3;
        const int z = 1 << (LV - l);
        int pw2[8] = {}, cf2[8] = {}, m2 = 0;
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
  u32* Q = k.prod + ((size_t)p * k.prod_tiles + lt) * tile_words(k.nwp);
  const long long* cb = k.m.carry + ((size_t)p * ntiles + lt) * rt.n * 1024 + e;
  for (int w = 0; w + 1 < rt.n; ++w) add_at_limb(Q, r, c, MF_LPB * rt.tb[w + 1], k.nwp, cb[(size_t)w * 1024]);
}

// a -= sum_p c_p(Y) P_p for every live entry of the launch, one thread per
// entry.  Y is O slabs, the entry 2^(L+1) segments of O slabs, every product
// 2 O + 1 slabs with a signed top slab.  Output slab m O + jj takes, from term
// (p, pw), product slab (m - pw) O + jj: slab jj for m = pw, O + jj for m = pw + 1,
// and the top slab 2 O at jj = 0 for m = pw + 2.  So the thread walks jj, holds
// slab jj of every segment in registers, streams the two slabs jj and O + jj of
// every product through once, and stores the segments, each with its own
// running carry; at the end the carry out of segment m enters at its
// successor's first slab.
__device__ __forceinline__ void ka_apply(i64* s, const uint4& v, int sg, bool top) {
  const i64 v3 = top ? (i64)(int)v.w : (i64)v.w;
  if (sg > 0) {
    s[0] += v.x; s[1] += v.y; s[2] += v.z; s[3] += v3;
  } else {
    s[0] -= v.x; s[1] -= v.y; s[2] -= v.z; s[3] -= v3;
  }
}

// Term TI onwards, every index a compile-time constant: the slabs of a product
// are loaded at its first term, products in groups of three whose loads are in
// flight together (the fence keeps the compiler from hoisting later groups'
// loads into registers the accumulators need).
// 16 bytes at the wave-uniform base plus the lane's byte offset (keeps the
// many product and segment bases in scalar registers)
__device__ __forceinline__ uint4 ld_lane(const u32* base, u32 voff) {
  return *(const uint4*)((const char*)base + voff);
}

// does product p have a term reaching segments [M0, M1)?
template <int LV>
constexpr bool ka_needed(int p, int M0, int M1) {
  const KaPoly<LV> T{};
  for (int t = T.first[p]; t < T.first[p + 1]; ++t)
    if (T.t[t].pw < M1 && T.t[t].pw + 2 >= M0) return true;
  return false;
}

// Term TI onwards for the segments [M0, M1) held in s (s[0] is segment M0),
// every index a compile-time constant: the slabs of a product are loaded at its
// first term, products in groups of three whose loads are in flight together
// (the fence keeps the compiler from hoisting later groups' loads into the
// registers the accumulators need).
template <int LV, int M0, int M1, int TI>
__device__ __forceinline__ void ka_term(i64 (&s)[M1 - M0][4], const u32* P0, u32& voff, size_t pst, int O, int jj,
                                        uint4& lo, uint4& hi, uint4& top) {
  constexpr KaTerm TT = KaPoly<LV>().t[TI];
  if constexpr (ka_needed<LV>(TT.p, M0, M1)) {
    if constexpr (TI == KaPoly<LV>().first[TT.p]) {
      // a new group of three products: its addresses take a (void) dependence
      // on every accumulator, so its loads issue after the previous group has
      // been added in and at most one group's slabs occupy registers
      if constexpr (TT.p % 3 == 0 && TT.p > 0) {
        u32 dep = 0;
#pragma unroll
        for (int m = 0; m < M1 - M0; ++m) dep ^= (u32)s[m][0] ^ (u32)s[m][1] ^ (u32)s[m][2] ^ (u32)s[m][3];
        asm volatile("" : "+v"(voff) : "v"(dep));
      }
      const u32* Qp = P0 + (size_t)TT.p * pst;
      lo = ld_lane(Qp + (size_t)jj * 4096, voff);
      hi = ld_lane(Qp + (size_t)(O + jj) * 4096, voff);
      if (jj == 0) top = ld_lane(Qp + (size_t)(2 * O) * 4096, voff);
    }
    if constexpr (TT.pw >= M0 && TT.pw < M1) ka_apply(s[TT.pw - M0], lo, TT.sg, false);
    if constexpr (TT.pw + 1 >= M0 && TT.pw + 1 < M1) ka_apply(s[TT.pw + 1 - M0], hi, TT.sg, false);
    if constexpr (TT.pw + 2 >= M0 && TT.pw + 2 < M1) {
      if (jj == 0) ka_apply(s[TT.pw + 2 - M0], top, TT.sg, true);
    }
  }
}

// every term, each a separate inlined call (no recursion, so the accumulators
// stay in registers)
template <int LV, int M0, int M1, int... TI>
__device__ __forceinline__ void ka_terms(std::integer_sequence<int, TI...>, i64 (&s)[M1 - M0][4], const u32* P0,
                                         u32& voff, size_t pst, int O, int jj) {
  uint4 lo = make_uint4(0u, 0u, 0u, 0u), hi = lo, top = lo;
  (ka_term<LV, M0, M1, TI>(s, P0, voff, pst, O, jj, lo, hi, top), ...);
}

// segments [M0, M1) of the entry: slab jj of each in registers, the products
// reaching them streamed through once per jj; cy[m - M0] is the carry out of
// segment m
template <int LV, int M0, int M1>
__device__ __forceinline__ void ka_pass(u32* At, const u32* P0, u32 voff0, size_t pst, int O, i64 (&cy)[M1 - M0]) {
  constexpr int NS = M1 - M0;
#pragma unroll
  for (int m = 0; m < NS; ++m) cy[m] = 0;
  for (int jj = 0; jj < O; ++jj) {
    u32 voff = voff0;
    i64 s[NS][4];
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const uint4 a = ld_lane(At + (size_t)((M0 + m) * O + jj) * 4096, voff);
      s[m][0] = a.x; s[m][1] = a.y; s[m][2] = a.z; s[m][3] = a.w;
    }
    ka_terms<LV, M0, M1>(std::make_integer_sequence<int, KaPoly<LV>::NT>{}, s, P0, voff, pst, O, jj);
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      i64 s0 = s[m][0] + cy[m], s1 = s[m][1], s2 = s[m][2], s3 = s[m][3];
      s1 += s0 >> 32;
      s2 += s1 >> 32;
      s3 += s2 >> 32;
      cy[m] = s3 >> 32;
      *(uint4*)((char*)(At + (size_t)((M0 + m) * O + jj) * 4096) + voff) =
          make_uint4((u32)s0, (u32)s1, (u32)s2, (u32)s3);
    }
  }
}

// a -= sum_p c_p(Y) P_p for every live entry of the launch, one thread per
// entry (see ka_pass), in passes of at most eight segments; then the carry out
// of every segment enters at its successor's first slab (the last one leaves
// the entry).
template <int LV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LV == 1 ? 4 : 2)))
void k_kara_comb(KaraArgs k, int C_lo) {
  constexpr int NSEG = 2 << LV;
  const UpdArgs& g = k.m.g;
  const int lt = blockIdx.x >> 2, e = (blockIdx.x & 3) * 256 + threadIdx.x;
  int R, C;
  if (!kara_entry(k, C_lo, lt, e, &R, &C) || has_error(g.st)) return;
  const int r = e >> 5, c = e & 31;
  const size_t tix = g.tri ? tri_tile_index(R, C) : (size_t)R * g.ntc + C;
  const size_t tw = tile_words(k.nwp), pst = k.prod_tiles * tw;
  u32* At = g.A + tix * tile_words(g.nw);   // wave-uniform bases, the lane's offset apart
  const u32* P0 = k.prod + (size_t)lt * tw;
  const u32 voff = (u32)in_tile(r, c, 0) * 4;
  const int O = k.m.S / (16 << LV);
  if constexpr (NSEG <= 16) {
    i64 cy[NSEG];
    ka_pass<LV, 0, NSEG>(At, P0, voff, pst, O, cy);
#pragma unroll
    for (int m = 0; m + 1 < NSEG; ++m) add_at_limb(At, r, c, 4 * (m + 1) * O, g.nw, cy[m]);
  } else {
    i64 cy0[8], cy1[NSEG - 8];
    ka_pass<LV, 0, 8>(At, P0, voff, pst, O, cy0);
    ka_pass<LV, 8, NSEG>(At, P0, voff, pst, O, cy1);
#pragma unroll
    for (int m = 0; m < 8; ++m) add_at_limb(At, r, c, 4 * (m + 1) * O, g.nw, cy0[m]);
#pragma unroll
    for (int m = 0; m + 1 < NSEG - 8; ++m) add_at_limb(At, r, c, 4 * (m + 9) * O, g.nw, cy1[m]);
  }
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

hipError_t launch_upd_kara(const KaraArgs& k, hipStream_t stream) {
  const MfmaArgs& m = k.m;
  const UpdArgs& g = m.g;
  if (g.r_hi <= g.r_lo || g.c_hi <= g.c_lo || g.npan <= 0) return hipSuccess;
  if (!g.tri || (g.rsb != 0 && g.rsb != (size_t)g.nl)) return hipErrorInvalidValue;
  const int L = k.levels, h = m.S / 2;
  if (L < 1 || L > KA_MAX_LEVELS) return hipErrorInvalidValue;
  const int np = kara_products(L);
  // the split points on whole 4-limb slabs, padding, 32-bit buffer offsets
  bool ok = m.S % (16 << L) == 0 && m.S == 4 * g.nl && k.Sk == kara_leaf_digits(m.S, L) &&
            k.nwp == kara_nwp(m.S, L) && m.pad >= MF_PAD_MIN && k.kslices == k.Sk + 2 * m.pad &&
            k.nwp / 4 == 2 * (m.S / (16 << L)) + 1;
  for (int l = 1; l <= L; ++l)
    ok = ok && k.pan[l] && k.pan_slices[l] == kara_leaf_digits(m.S, l) + 2 * m.pad &&
         (size_t)k.pan_slices[l] * m.NT * 16 <= 0x7fffffffu && k.pan_stride[l] >= (size_t)k.pan_slices[l] * m.NT * 16;
  if (!ok) return hipErrorInvalidValue;
  const size_t rthreads = (size_t)g.nl * m.NT * 16;
  const unsigned rblocks = (unsigned)((rthreads + 255) / 256);
  int8_t* l1[6];
  for (int q = 0; q < 6; ++q) l1[q] = k.pan[1] + (size_t)q * k.pan_stride[1];
  hipLaunchKernelGGL(k_recode_kara, dim3(rblocks), dim3(256), 0, stream, g.Bop, g.ldb, g.npan, m.NT, m.NT, g.nl,
                     m.pad, h / 4, l1[0], l1[1]);
  hipLaunchKernelGGL(k_recode_kara, dim3(rblocks), dim3(256), 0, stream, g.Uop, g.ldu, g.npan, m.NT, m.u_rows,
                     g.nl, m.pad, h / 4, l1[3], l1[4]);
  {
    const size_t threads = (size_t)(h / 4 + 1) * m.NT * 16;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    hipLaunchKernelGGL(k_kara_mid, dim3(blocks), dim3(256), 0, stream, l1[0], l1[1], m.NT, m.pad, h, l1[2]);
    hipLaunchKernelGGL(k_kara_mid, dim3(blocks), dim3(256), 0, stream, l1[3], l1[4], m.NT, m.pad, h, l1[5]);
  }
  for (int l = 2; l <= L; ++l) {
    // every level-(l-1) panel (at most S/2^(l-1) + l - 1 digits) splits at S/2^l
    const int nmax = (m.S >> (l - 1)) + l - 1, s = m.S >> l, parents = 2 * kara_products(l - 1);
    const size_t threads = (size_t)nmax * m.NT;
    hipLaunchKernelGGL(k_digit_split, dim3((unsigned)((threads + 255) / 256), parents), dim3(256), 0, stream, k, l);
    const size_t mthreads = (size_t)((s + l - 1) / 4 + 1) * m.NT * 16;
    hipLaunchKernelGGL(k_kara_mid_lv, dim3((unsigned)((mthreads + 255) / 256), parents), dim3(256), 0, stream, k, l);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
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
  hipLaunchKernelGGL(k_upd_kara, dim3(8 * per_xcd), dim3(64), 0, stream, k, rt, C_lo, ntiles, per_xcd);
  e = hipGetLastError();
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
  if (rt.n > 1) hipLaunchKernelGGL(k_kara_fix, dim3(4 * ntiles, np), dim3(256), 0, stream, k, rt, C_lo, ntiles);
  if (L == 1)
    hipLaunchKernelGGL(k_kara_comb<1>, dim3(4 * ntiles), dim3(256), 0, stream, k, C_lo);
  else if (L == 2)
    hipLaunchKernelGGL(k_kara_comb<2>, dim3(4 * ntiles), dim3(256), 0, stream, k, C_lo);
  else
    hipLaunchKernelGGL(k_kara_comb<3>, dim3(4 * ntiles), dim3(256), 0, stream, k, C_lo);
  e = hipGetLastError();
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
