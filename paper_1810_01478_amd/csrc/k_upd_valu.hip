// Exact Schur-complement update on the vector ALU (the "plain" form):
//   A[r][c] <- A[r][c] - sum_{i in panel} b_ri u_ci        (Algorithm 1, inner loops)
// with b, u two's complement P-bit numbers (nl limbs) and A a 2P-bit two's
// complement number (nw = 2 nl limbs); the arithmetic is exact modulo 2^(32 nw),
// which gives the exact result because the true result fits in nw limbs.
//
// One wave per target entry.  Lane l owns output columns t = l + 64 q
// (q = 0..Q-1) and accumulates sum_x b[x] u[t-x] in 96 bits per column with
// v_mad_u64_u32 (32 x 32 -> 64-bit multiply-add) and a carry count.  Both
// factors of the current panel column sit in LDS; for t < nl all lanes read the
// same b[x] (broadcast) and consecutive u[t-x], for t >= nl the reverse, so the
// reads are free of bank conflicts.
//
// Signs: for two's complement x, y over nl limbs,
//   x y = x_u y_u - 2^(32 nl) (s_x y_u + s_y x_u)   (mod 2^(64 nl)),
// and -Y 2^(32 nl) = (~Y + 1) 2^(32 nl) (mod 2^(64 nl)) with ~Y over nl limbs, so
// the sign terms are added as complemented limbs in the upper columns.
// The subtraction uses a - S = ~(~a + S): the accumulators start from the
// complemented limbs of a and the resolved sum is complemented on the way out.
#include "hl_kernels.hpp"

namespace hl {

__device__ __forceinline__ u32* entry_base(const UpdArgs& g, int r, int c) {
  size_t t = g.tri ? tri_tile_index(r >> 5, c >> 5) : (size_t)(r >> 5) * g.ntc + (c >> 5);
  return g.A + t * tile_words(g.nw);
}

template <int Q>
__device__ void upd_valu_body(const UpdArgs& g, int bx, int by) {
  const int r = g.r_lo + bx;
  const int c = g.c_lo + by;
  if (r >= g.r_hi || c >= g.c_hi) return;
  if (g.tri && r < c) return;
  if (has_error(g.st)) return;
  extern __shared__ u32 sm[];
  const int nl = g.nl, nw = g.nw;
  u32* sb = sm;
  u32* su = sm + nl;
  const int l = lane_id();
  u32* Ab = entry_base(g, r, c);
  u64 lo[Q];
  u32 hi[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int t = l + WAVE * q;
    lo[q] = (t < nw) ? (u64)(~Ab[in_tile(r, c, t)]) : 0ull;
    hi[q] = 0;
  }
  for (int il = 0; il < g.npan; ++il) {
    const u32* bp = g.Bop + (size_t)il * g.ldb + (size_t)r * (g.rsb ? g.rsb : (size_t)nl);
    const u32* up = g.Uop + (size_t)il * g.ldu + (size_t)c * nl;
    __syncthreads();
    for (int p = l; p < nl; p += WAVE) {
      sb[p] = bp[p];
      su[p] = up[p];
    }
    __syncthreads();
    const u32 sgb = sb[nl - 1] >> 31, sgu = su[nl - 1] >> 31;
    // keep the per-column bounds inside the panel loop (hoisting them costs
    // several registers per column)
    int lane = l;
    asm volatile("" : "+v"(lane));
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int t = lane + WAVE * q;
      if (t < 2 * nl - 1) {
        const int x0 = t - nl + 1 > 0 ? t - nl + 1 : 0;
        const int x1 = t < nl - 1 ? t : nl - 1;
        col_sum(sb, su, t, x0, x1, lo[q], hi[q]);
      }
      if (t >= nl && t < 2 * nl) {
        u64 s = 0;
        if (sgb) s += (u64)(~su[t - nl]);
        if (sgu) s += (u64)(~sb[t - nl]);
        if (t == nl) s += (u64)(sgb + sgu);
        const u64 n2 = lo[q] + s;
        hi[q] += (n2 < s) ? 1u : 0u;
        lo[q] = n2;
      }
    }
  }
  // resolve 64 columns at a time and store the complemented limbs
  u32 carry = 0, sp_mid = 0, sp62 = 0, sp63 = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const u32 w0 = (u32)lo[q], w1 = (u32)(lo[q] >> 32), w2 = hi[q];
    u32 m1 = shfl_up_u32(w1, 1);
    u32 h2 = shfl_up_u32(w2, 2);
    if (l == 0) {
      m1 = sp_mid;
      h2 = sp62;
    }
    if (l == 1) h2 = sp63;
    const u64 v = (u64)w0 + m1 + h2;
    const u32 limb = w_resolve(v, carry);
    const int t = l + WAVE * q;
    if (t < nw) Ab[in_tile(r, c, t)] = ~limb;
    sp_mid = shfl_u32(w1, WAVE - 1);
    sp62 = shfl_u32(w2, WAVE - 2);
    sp63 = shfl_u32(w2, WAVE - 1);
  }
}

template <int Q>
__global__ __launch_bounds__(64) void k_upd_valu(UpdArgs g) {
  upd_valu_body<Q>(g, blockIdx.x, blockIdx.y);
}

// Workgroup form for launches with few entries: VW waves per entry, wave w
// owning the 64-column chunks w, w + VW, ...; the 96-bit column sums meet in
// LDS and wave 0 resolves them into limbs (as g_mul does).  Same result bits.
constexpr int VW = 4;

template <int QW>
__global__ __launch_bounds__(VW * 64) void k_upd_valu_wg(UpdArgs g) {
  const int r = g.r_lo + blockIdx.x;
  const int c = g.c_lo + blockIdx.y;
  if (r >= g.r_hi || c >= g.c_hi) return;
  if (g.tri && r < c) return;
  if (has_error(g.st)) return;
  extern __shared__ u32 sm[];
  const int nl = g.nl, nw = g.nw;
  const int Qn = (nw + WAVE - 1) / WAVE;
  u32* sb = sm;
  u32* su = sm + nl;
  u32* cs = sm + 2 * nl;  // 3 words per column, 64 Qn columns
  const int l = lane_id(), w = wave_id();
  u32* Ab = entry_base(g, r, c);
  u64 lo[QW];
  u32 hi[QW];
#pragma unroll
  for (int i = 0; i < QW; ++i) {
    const int t = WAVE * (w + VW * i) + l;
    lo[i] = (t < nw) ? (u64)(~Ab[in_tile(r, c, t)]) : 0ull;
    hi[i] = 0;
  }
  for (int il = 0; il < g.npan; ++il) {
    const u32* bp = g.Bop + (size_t)il * g.ldb + (size_t)r * (g.rsb ? g.rsb : (size_t)nl);
    const u32* up = g.Uop + (size_t)il * g.ldu + (size_t)c * nl;
    __syncthreads();
    for (int p = threadIdx.x; p < nl; p += blockDim.x) {
      sb[p] = bp[p];
      su[p] = up[p];
    }
    __syncthreads();
    const u32 sgb = sb[nl - 1] >> 31, sgu = su[nl - 1] >> 31;
    int lane = l;
    asm volatile("" : "+v"(lane));
#pragma unroll
    for (int i = 0; i < QW; ++i) {
      const int t = lane + WAVE * (w + VW * i);
      if (t < 2 * nl - 1) {
        const int x0 = t - nl + 1 > 0 ? t - nl + 1 : 0;
        const int x1 = t < nl - 1 ? t : nl - 1;
        col_sum(sb, su, t, x0, x1, lo[i], hi[i]);
      }
      if (t >= nl && t < 2 * nl) {
        u64 s2 = 0;
        if (sgb) s2 += (u64)(~su[t - nl]);
        if (sgu) s2 += (u64)(~sb[t - nl]);
        if (t == nl) s2 += (u64)(sgb + sgu);
        const u64 n2 = lo[i] + s2;
        hi[i] += (n2 < s2) ? 1u : 0u;
        lo[i] = n2;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < QW; ++i) {
    const int t = WAVE * (w + VW * i) + l;
    if (t < WAVE * Qn) {
      cs[3 * t] = (u32)lo[i];
      cs[3 * t + 1] = (u32)(lo[i] >> 32);
      cs[3 * t + 2] = hi[i];
    }
  }
  __syncthreads();
  if (w == 0) {
    u32 carry = 0;
    for (int ch = 0; ch < Qn; ++ch) {
      const int p = ch * WAVE + l;
      u64 v = cs[3 * p];
      if (p >= 1) v += cs[3 * (p - 1) + 1];
      if (p >= 2) v += cs[3 * (p - 2) + 2];
      const u32 limb = w_resolve(v, carry);
      if (p < nw) Ab[in_tile(r, c, p)] = ~limb;
    }
  }
}

template <int QW>
static hipError_t launch_wg(const UpdArgs& g, hipStream_t stream) {
  const int nr = g.r_hi - g.r_lo, nc = g.c_hi - g.c_lo;
  const int Qn = (g.nw + WAVE - 1) / WAVE;
  const size_t lds = ((size_t)2 * g.nl + (size_t)3 * WAVE * Qn) * 4;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_upd_valu_wg<QW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_upd_valu_wg<QW>, dim3(nr, nc), dim3(VW * 64), lds, stream, g);
  return hipGetLastError();
}

static hipError_t launch_wg_any(const UpdArgs& g, hipStream_t stream) {
  const int Qn = (g.nw + WAVE - 1) / WAVE;
  const int QW = (Qn + VW - 1) / VW;
  if (QW <= 2) return launch_wg<2>(g, stream);
  if (QW <= 3) return launch_wg<3>(g, stream);
  if (QW <= 4) return launch_wg<4>(g, stream);
  if (QW <= 6) return launch_wg<6>(g, stream);
  if (QW <= 8) return launch_wg<8>(g, stream);
  if (QW <= 10) return launch_wg<10>(g, stream);
  if (QW <= 12) return launch_wg<12>(g, stream);
  if (QW <= 14) return launch_wg<14>(g, stream);
  return launch_wg<16>(g, stream);
}

// batch: blockIdx.z is the instance; every record fits Q
template <int Q>
__global__ __launch_bounds__(64) void k_upd_valu_b(const UpdArgs* __restrict__ tab) {
  upd_valu_body<Q>(tab[blockIdx.z], blockIdx.x, blockIdx.y);
}

// one launch of either form: g != nullptr (single record by value) or tab
template <int Q>
static hipError_t launch_q(const UpdArgs* g, const UpdArgs* tab, int count, int nr, int nc, int nl,
                           hipStream_t stream) {
  if (nr <= 0 || nc <= 0 || count <= 0) return hipSuccess;
  const size_t lds = (size_t)2 * nl * 4;
  if (g)
    hipLaunchKernelGGL(k_upd_valu<Q>, dim3(nr, nc), dim3(64), lds, stream, *g);
  else
    hipLaunchKernelGGL(k_upd_valu_b<Q>, dim3(nr, nc, count), dim3(64), lds, stream, tab);
  return hipGetLastError();
}

static hipError_t launch_any(const UpdArgs* g, const UpdArgs* tab, int count, int nr, int nc, int nw, int nl,
                             hipStream_t stream) {
  const int Qn = (nw + WAVE - 1) / WAVE;
  if (Qn <= 1) return launch_q<1>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 2) return launch_q<2>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 3) return launch_q<3>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 4) return launch_q<4>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 6) return launch_q<6>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 8) return launch_q<8>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 10) return launch_q<10>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 12) return launch_q<12>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 16) return launch_q<16>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 20) return launch_q<20>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 24) return launch_q<24>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 32) return launch_q<32>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 40) return launch_q<40>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 48) return launch_q<48>(g, tab, count, nr, nc, nl, stream);
  if (Qn <= 56) return launch_q<56>(g, tab, count, nr, nc, nl, stream);
  return launch_q<64>(g, tab, count, nr, nc, nl, stream);
}

hipError_t launch_upd_valu(const UpdArgs& g, hipStream_t stream) {
  if (g.npan <= 0) return hipSuccess;
  const int nr = g.r_hi - g.r_lo, nc = g.c_hi - g.c_lo;
  if (nr <= 0 || nc <= 0) return hipSuccess;
  // few entries of long numbers: one wave per entry would leave most SIMDs idle
  const int Qn = (g.nw + WAVE - 1) / WAVE;
  if ((long)nr * nc < 1536 && Qn >= 8) return launch_wg_any(g, stream);
  return launch_any(&g, nullptr, 1, nr, nc, g.nw, g.nl, stream);
}

// ---------------------------------------------------------------------------
// Issue-rate probe of the vector ALU's integer multiply-add (the plain form's
// limb product): every lane runs 8 independent chains of iters steps, either
// the plain form's pair (v_mad_u64_u32 into a 64-bit accumulator and
// v_addc_co_u32 of its carry into a count, MODE 0) or v_mad_u64_u32 alone
// (MODE 1).  Operands stay in registers, so nothing but the ALU is measured.
template <int MODE>
__global__ __launch_bounds__(256) void k_valu_peak(int iters, u64* sink) {
  const u32 b = threadIdx.x * 2654435761u + blockIdx.x;
  u64 lo[8];
  u32 hi[8], a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    lo[k] = k;
    hi[k] = 0;
    a[k] = (b ^ (0x9e3779b9u * (k + 1))) | 1u;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (MODE == 0)
        mac96(lo[k], hi[k], a[k], b);
      else
        asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(lo[k]) : "v"(a[k]), "v"(b) : "vcc");
    }
  }
  u64 s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += lo[k] + hi[k];
  if (s == 0x0123456789abcdefull) sink[0] = s;  // keeps the chains live
}

hipError_t launch_valu_peak(int mode, int blocks, int iters, u64* sink, hipStream_t stream) {
  if (mode == 0)
    hipLaunchKernelGGL(k_valu_peak<0>, dim3(blocks), dim3(256), 0, stream, iters, sink);
  else
    hipLaunchKernelGGL(k_valu_peak<1>, dim3(blocks), dim3(256), 0, stream, iters, sink);
  return hipGetLastError();
}

hipError_t launch_upd_valu_batch(const UpdArgs* tab, int count, int nr_max, int nc_max, int nw_max, int nl_max,
                                 hipStream_t stream) {
  return launch_any(nullptr, tab, count, nr_max, nc_max, nw_max, nl_max, stream);
}

}  // namespace hl
