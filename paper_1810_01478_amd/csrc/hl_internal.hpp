// Internal layouts shared by the kernels and the host orchestration.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/hl.h"

namespace hl {

// status word in device memory (first 16 bytes of the workspace)
struct DevStatus {
  unsigned long long code_index;  // (code << 32) | index, first error wins
  int flags[2];
};

__device__ __forceinline__ void set_status(DevStatus* st, int code, int index) {
  unsigned long long v = ((unsigned long long)(unsigned)code << 32) | (unsigned)index;
  atomicCAS(&st->code_index, 0ull, v);
}
__device__ __forceinline__ bool has_error(const DevStatus* st) {
  return *((volatile const unsigned long long*)&st->code_index) != 0ull;
}

// deepest Karatsuba level of the Schur update (3^4 = 81 digit-sum products)
constexpr int KA_MAX_LEVELS = 4;

// Sizes derived from a shape.
struct Dims {
  int N;         // order
  int NT;        // N rounded up to a multiple of 32
  int nt;        // NT / 32 (tile rows)
  int P;         // precision bits (multiple of 128)
  int nl;        // P / 32 limbs per factor-sized number
  int nw;        // 2 * nl limbs per trailing entry
  int S;         // 4 * nl signed 8-bit digits per factor
  int E;         // exponent block
  int k;
  int W;         // 2P - 4
  int kara;      // Karatsuba levels of the Schur update available (MFMA form): 0 .. 4
  int Sk0;       // digits of a factor in the Karatsuba form: S rounded up to a multiple of 256
                 // (zero digits on top), so every level splits on whole 16-digit slabs
};

// Trailing matrix: 32 x 32 tiles (R >= C) packed row by row; inside a tile the
// entries are grouped in 4-limb (16-byte) slabs: [slab q][r][c][4].
__host__ __device__ __forceinline__ size_t tri_tile_index(int R, int C) {
  return (size_t)R * (R + 1) / 2 + C;
}
__host__ __device__ __forceinline__ size_t tile_words(int nw) { return (size_t)nw * 1024; }

// word offset of limb l of entry (r, c) inside a tile
__host__ __device__ __forceinline__ size_t in_tile(int r, int c, int l) {
  return ((size_t)(l >> 2) * 1024 + (size_t)(r & 31) * 32 + (c & 31)) * 4 + (l & 3);
}

// Target description for the exact update A[r][c] -= sum_i b_ri u_ci.
struct UpdArgs {
  uint32_t* A;           // tile storage
  int tri;               // 1: lower triangular tile packing, 0: rectangular
  int ntc;               // tile columns (rectangular packing)
  int nw;                // limbs per entry (2 nl)
  int nl;                // limbs per factor
  const uint32_t* Bop;   // b_ri at Bop + il*ldb + r*rsb  (two's complement, nl limbs)
  size_t ldb;
  size_t rsb;            // row stride of Bop in limbs (0: nl); the MFMA form needs nl
  const uint32_t* Uop;   // u_ci at Uop + il*ldu + c*nl
  size_t ldu;
  int npan;              // number of factor columns i (<= 16)
  int r_lo, r_hi;        // rows updated: [r_lo, r_hi)
  int c_lo, c_hi;        // columns updated: [c_lo, c_hi); tri also needs r >= c
  DevStatus* st;
};

}  // namespace hl
