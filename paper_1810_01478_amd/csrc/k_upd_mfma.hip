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
// digits are taken 8 at a time (8 accumulators of 16 registers); for the 8
// accumulators of one step the B operands are 8 consecutive digit slices, and
// the next step (j0 + 2) needs the same slices shifted by two, so a window of
// 10 slices rotates through registers and each step loads one A slice and two
// new B slices for eight MFMAs.  Digit slices outside [0, S) are zero padding.
//
// Recombination.  After the j loop of 8 output digits (2 limbs), each lane folds
// its 16 entries: X = A[2 limbs] - sum_q out_(t0+q) 256^q + carry, an exact
// 128-bit value; the low 64 bits are the new limbs and X >> 64 the carry into
// the next pair of limbs.  The carry out of each wave's limb range is stored
// and added by k_carry_fix, so ranges of one tile run in parallel.
#include "hl_kernels.hpp"

namespace hl {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int MF_T = 8;  // output digits per accumulation block (2 limbs)

struct RangeTab {
  int n;        // ranges
  int tb[17];   // t-block boundaries, tb[0] = 0, tb[n] = nl
};

// entry (m, n) of the 32 x 32 MFMA result held by lane l, register v
__device__ __forceinline__ int mf_row(int l, int v) { return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3); }
__device__ __forceinline__ int mf_col(int l) { return l & 31; }

// ---------------------------------------------------------------------------
// Recode the panel factors (two's complement, nl limbs) into balanced digits.
// src: [16][NT][nl] limbs; dst: [slices][NT][16] bytes, slice = digit + pad.
__global__ void k_recode(const u32* __restrict__ src, size_t lds, int npan, int NT, int nrows, int nl, int pad,
                         int8_t* __restrict__ dst) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int il = gid & 15, row = gid >> 4;
  if (row >= NT) return;
  const int S = 4 * nl;
  const size_t rstride = (size_t)NT * 16;
  int8_t* d = dst + (size_t)pad * rstride + (size_t)row * 16 + il;
  if (il >= npan || row >= nrows) {
    for (int j = 0; j < S; ++j) d[(size_t)j * rstride] = 0;
    return;
  }
  const u32* x = src + (size_t)il * lds + (size_t)row * nl;
  int carry = 0;
  for (int q = 0; q < nl; ++q) {
    const u32 limb = x[q];
    for (int b = 0; b < 4; ++b) {
      const int j = 4 * q + b;
      int v;
      if (j == S - 1)
        v = (int)(int8_t)(limb >> 24) + carry;
      else
        v = (int)((limb >> (8 * b)) & 0xffu) + carry;
      if (j < S - 1 && v >= 128) {
        v -= 256;
        carry = 1;
      } else {
        carry = 0;
      }
      d[(size_t)j * rstride] = (int8_t)v;
    }
  }
}

__device__ __forceinline__ v4i ld16(const int8_t* p) { return *(const v4i*)p; }

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_upd_mfma(MfmaArgs m, RangeTab rt, int C_lo) {
  const UpdArgs& g = m.g;
  // triangular target: tiles (R, C), C_lo <= C <= R; rectangular: rows from
  // C_lo (here the first tile row), all g.ntc tile columns
  const int R = C_lo + blockIdx.x, C = g.tri ? C_lo + blockIdx.y : blockIdx.y, rg = blockIdx.z;
  if ((g.tri && R < C) || R * 32 >= m.NT) return;
  const size_t tix = g.tri ? tri_tile_index(R, C) : (size_t)R * g.ntc + C;
  if (has_error(g.st)) return;
  __shared__ i64 carry_s[16 * WAVE];  // carry of each of the lane's 16 entries
  const int l = lane_id(), h = l >> 5, mm = l & 31;
  const int S = m.S, NT = m.NT, pad = m.pad;
  const long sstride = (long)NT * 16;  // bytes per digit slice
  // A operand (b digits of tile rows), B operand (u digits of tile columns)
  const int8_t* Ab = m.bdig + (long)(pad + h) * sstride + (long)(R * 32 + mm) * 16;
  const int8_t* Ub = m.udig + (long)(pad - h) * sstride + (long)(C * 32 + mm) * 16;
  u32* At = g.A + tix * tile_words(g.nw);
  unsigned live = 0;  // entries of the trailing matrix proper (r >= c, inside the target)
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    carry_s[v * WAVE + l] = 0;
    const int r = R * 32 + mf_row(l, v), c = C * 32 + mf_col(l);
    if ((!g.tri || r >= c) && r >= g.r_lo && r < g.r_hi && c >= g.c_lo && c < g.c_hi) live |= 1u << v;
  }
  const int tb0 = rt.tb[rg], tb1 = rt.tb[rg + 1];
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
    const int nrot = (nsteps + 4) / 5;
    // window: slice x = t0 + q - j0 - h sits at Ub + (t0 + q - j0) * sstride
    const int8_t* ub0 = Ub + (long)(t0 - jlo) * sstride;
    v4i w0 = ld16(ub0 + 0 * sstride), w1 = ld16(ub0 + 1 * sstride), w2 = ld16(ub0 + 2 * sstride),
        w3 = ld16(ub0 + 3 * sstride), w4 = ld16(ub0 + 4 * sstride), w5 = ld16(ub0 + 5 * sstride),
        w6 = ld16(ub0 + 6 * sstride), w7 = ld16(ub0 + 7 * sstride), w8, w9;
    const int8_t* ap = Ab + (long)jlo * sstride;
    const int8_t* un = ub0 - 2 * sstride;  // next window's slices 0, 1
    v4i an = ld16(ap);                    // A of the current step, loaded one step ahead
#define MF_STEP(P0, P1, P2, P3, P4, P5, P6, P7, N0, N1)                                   \
  {                                                                                       \
    const v4i a = an;                                                                     \
    an = ld16(ap + 2 * sstride);                                                          \
    N0 = ld16(un);                                                                        \
    N1 = ld16(un + sstride);                                                              \
    acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, P0, acc[0], 0, 0, 0);               \
    acc[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, P1, acc[1], 0, 0, 0);               \
    acc[2] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, P2, acc[2], 0, 0, 0);               \
    acc[3] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, P3, acc[3], 0, 0, 0);               \
    acc[4] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, P4, acc[4], 0, 0, 0);               \
    acc[5] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, P5, acc[5], 0, 0, 0);               \
    acc[6] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, P6, acc[6], 0, 0, 0);               \
    acc[7] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, P7, acc[7], 0, 0, 0);               \
    ap += 2 * sstride;                                                                    \
    un -= 2 * sstride;                                                                    \
    __builtin_amdgcn_sched_group_barrier(0x020, 3, 0);                                    \
    __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);                                    \
  }
    for (int rot = 0; rot < nrot; ++rot) {
      MF_STEP(w0, w1, w2, w3, w4, w5, w6, w7, w8, w9)
      MF_STEP(w8, w9, w0, w1, w2, w3, w4, w5, w6, w7)
      MF_STEP(w6, w7, w8, w9, w0, w1, w2, w3, w4, w5)
      MF_STEP(w4, w5, w6, w7, w8, w9, w0, w1, w2, w3)
      MF_STEP(w2, w3, w4, w5, w6, w7, w8, w9, w0, w1)
    }
#undef MF_STEP
    // fold the 8 digit sums of each entry into limbs 2 tb, 2 tb + 1
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      if (!((live >> v) & 1u)) continue;
      const int r = mf_row(l, v), c = mf_col(l);
      u32* p = At + in_tile(r, c, 2 * tb);
      const u64 a64 = ((u64)p[1] << 32) | p[0];
      i64 vlo = 0, vhi = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) vlo += (i64)acc[q][v] << (8 * q);
#pragma unroll
      for (int q = 4; q < 8; ++q) vhi += (i64)acc[q][v] << (8 * (q - 4));
      __int128 X = (__int128)a64 - (__int128)vlo - ((__int128)vhi << 32) + (__int128)carry_s[v * WAVE + l];
      const u64 nl64 = (u64)X;
      p[0] = (u32)nl64;
      p[1] = (u32)(nl64 >> 32);
      carry_s[v * WAVE + l] = (i64)(X >> 64);
    }
  }
  // carries out of this range
  long long* cb = m.carry + (tix * (size_t)m.max_ranges + rg) * 1024;
#pragma unroll
  for (int v = 0; v < 16; ++v) cb[mf_row(l, v) * 32 + mf_col(l)] = carry_s[v * WAVE + l];
}

// Add the carries of range w at limb 2 tb[w+1] of every entry, w = 0..n-2.
__global__ void k_carry_fix(MfmaArgs m, RangeTab rt, int C_lo) {
  const UpdArgs& g = m.g;
  const int R = C_lo + blockIdx.x, C = g.tri ? C_lo + blockIdx.y : blockIdx.y;
  if ((g.tri && R < C) || R * 32 >= m.NT) return;
  if (has_error(g.st)) return;
  const size_t tix = g.tri ? tri_tile_index(R, C) : (size_t)R * g.ntc + C;
  const int e = threadIdx.x;  // 0..1023
  const int r = e >> 5, c = e & 31;
  {
    const int rg = R * 32 + r, cg = C * 32 + c;
    if (!((!g.tri || rg >= cg) && rg >= g.r_lo && rg < g.r_hi && cg >= g.c_lo && cg < g.c_hi)) return;
  }
  u32* At = g.A + tix * tile_words(g.nw);
  const long long* cb = m.carry + tix * (size_t)m.max_ranges * 1024;
  const int nw = m.g.nw;
  for (int w = 0; w + 1 < rt.n; ++w) {
    const i64 cv = cb[(size_t)w * 1024 + e];
    if (cv == 0) continue;
    int li = 2 * rt.tb[w + 1];
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
static RangeTab make_ranges(int nl, int S, int ntiles) {
  // t-blocks tb = 0..nl-1 cover digits 8 tb .. 8 tb + 7; work ~ number of (t, j) pairs
  RangeTab rt{};
  int want = (4096 + ntiles - 1) / (ntiles > 0 ? ntiles : 1);
  if (want < 1) want = 1;
  if (want > 16) want = 16;
  if (want > nl) want = nl;
  double total = 0;
  for (int tb = 0; tb < nl; ++tb)
    for (int q = 0; q < MF_T; ++q) {
      const int t = MF_T * tb + q;
      int cnt = t + 1;
      if (cnt > S) cnt = S;
      if (2 * S - 1 - t < cnt) cnt = 2 * S - 1 - t;
      if (cnt > 0) total += cnt;
    }
  rt.n = want;
  rt.tb[0] = 0;
  double acc = 0;
  int k = 1;
  for (int tb = 0; tb < nl && k < want; ++tb) {
    for (int q = 0; q < MF_T; ++q) {
      const int t = MF_T * tb + q;
      int cnt = t + 1;
      if (cnt > S) cnt = S;
      if (2 * S - 1 - t < cnt) cnt = 2 * S - 1 - t;
      if (cnt > 0) acc += cnt;
    }
    if (acc >= total * k / want) rt.tb[k++] = tb + 1;
  }
  while (k < want) rt.tb[k++] = nl;
  rt.tb[want] = nl;
  // drop empty ranges
  int w = 1;
  for (int j = 1; j <= want; ++j)
    if (rt.tb[j] > rt.tb[w - 1]) rt.tb[w++] = rt.tb[j];
  rt.n = w - 1;
  return rt;
}

hipError_t launch_recode(const u32* src, size_t lds, int npan, int NT, int nrows, int nl, int pad, int8_t* dst,
                         hipStream_t stream) {
  const int threads = NT * 16;
  hipLaunchKernelGGL(k_recode, dim3((threads + 255) / 256), dim3(256), 0, stream, src, lds, npan, NT, nrows, nl,
                     pad, dst);
  return hipGetLastError();
}

hipError_t launch_upd_mfma(const MfmaArgs& m, hipStream_t stream) {
  const UpdArgs& g = m.g;
  if (g.r_hi <= g.r_lo || g.c_hi <= g.c_lo || g.npan <= 0) return hipSuccess;
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
  RangeTab rt = make_ranges(g.nl, m.S, ntiles);
  if (rt.n > m.max_ranges) return hipErrorInvalidValue;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (m.timing) {
    (void)hipEventCreate(&ev0);
    (void)hipEventCreate(&ev1);
    (void)hipEventRecord(ev0, stream);
  }
  hipLaunchKernelGGL(k_upd_mfma, dim3(nrow, ncol, rt.n), dim3(64), 0, stream, m, rt, C_lo);
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

hipError_t launch_mfma_probe(int* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, stream, out);
  return hipGetLastError();
}

}  // namespace hl
