// Kernel launchers shared between the kernel files and the host API.
#pragma once
#include <climits>
#include "mp.hpp"
#include "hl_internal.hpp"

namespace hl {

size_t pivot_lds_bytes(int nl);
size_t col_lds_bytes(int nl);

hipError_t launch_scales(const u32* mu, const i64* mu_exp, int w, int N, int E, i32* s, DevStatus* st,
                         hipStream_t stream);
hipError_t launch_load(const u32* mu, const i64* mu_exp, int w, const i32* s, const Dims& dm, u32* A,
                       DevStatus* st, hipStream_t stream);
hipError_t launch_pivot(u32* A, const Dims& dm, int i, u32* d_out, i32* h_out, u32* omega, int ostride,
                        DevStatus* st, hipStream_t stream, const u32* sub_b = nullptr, const u32* sub_u = nullptr,
                        int from_row = 0);
hipError_t launch_col(const u32* A, const Dims& dm, int i, int r0, const i32* h, const u32* omega,
                      int ostride, u32* u_out, u32* l_col, DevStatus* st, hipStream_t stream);
hipError_t launch_fill(u32* p, size_t n, u32 v, hipStream_t stream);
// the column step in one launch with the workgroup int8 MFMA product per row
// (hipErrorInvalidValue when its LDS would exceed 160 KiB)
hipError_t launch_col_m(const u32* A, const Dims& dm, int i, int r0, const i32* h, const u32* omega,
                        int ostride, u32* u_out, u32* l_col, DevStatus* st, hipStream_t stream);
// the column step split around an MFMA product (see k_col_u, k_col_fin)
hipError_t launch_col_u(const u32* A, const Dims& dm, int i, int r0, const i32* h, u32* u_out, DevStatus* st,
                        hipStream_t stream);
hipError_t launch_col_fin(const Dims& dm, int i, int r0, const u32* P, int ldp, u32* l_col, DevStatus* st,
                          hipStream_t stream);

// Argument records of the per-pivot kernels; a batch launch takes a device array
// of them, one per instance.
struct PivotArgs {
  u32* A;
  Dims dm;
  int i;
  u32* d_out;
  i32* h_out;
  u32* omega;
  int ostride;
  DevStatus* st;
  // optional (both or neither): the pivot is a_ii - sub_b sub_u, the previous
  // column's update of the diagonal entry, which the caller left out of that
  // column's in-panel update (nl limbs each, two's complement)
  const u32* sub_b = nullptr;
  const u32* sub_u = nullptr;
  // nonzero (with no sub_b, sub_u): the pivot is a_ii - b u with b, u the
  // previous column's factors of row i, formed here from a_(i,i-1), h_(i-1)
  // and w_(i-1) exactly as the column step forms them (so it need not wait for
  // that column step)
  int from_row = 0;
};
struct ColArgs {
  const u32* A;
  Dims dm;
  int i, r0;
  const i32* h;
  const u32* omega;
  int ostride;
  u32* u_out;
  u32* l_col;
  DevStatus* st;
};
hipError_t launch_pivot_batch(const PivotArgs* tab, int count, int nl_max, hipStream_t stream);
// batched split column step (one record per instance)
struct ColFinArgs {
  ColArgs c;
  const u32* P;  // products u_r w_i, rows ldp limbs apart
  int ldp;
};
hipError_t launch_col_u_batch(const ColArgs* tab, int count, int rows_max, int nl_max, hipStream_t stream);
hipError_t launch_col_fin_batch(const ColFinArgs* tab, int count, int rows_max, int ldp_max, hipStream_t stream);
hipError_t launch_col_batch(const ColArgs* tab, int count, int rows_max, int nl_max, hipStream_t stream);
hipError_t launch_debug_mul(const u32* a, int na, const u32* b, int nb, u32* out, int nout,
                            hipStream_t stream);
hipError_t launch_debug_recip(const u32* d, int nd, int P, u32* omega, int n_omega, i32* h,
                              hipStream_t stream);
// VALU multiply-add issue-rate probe (mode 0: v_mad_u64_u32 + carry count, 1: v_mad_u64_u32)
hipError_t launch_valu_peak(int mode, int blocks, int iters, u64* sink, hipStream_t stream);
hipError_t launch_debug_mul_wg(const u32* a, int na, const u32* b, int nb, u32* out, int nout, int threads,
                               hipStream_t stream);

// exact update A[r][c] -= sum_i b_ri u_ci on the vector ALU; the batch form
// takes a device array of records (grid nr_max x nc_max x count, each record
// bounded by its own row and column ranges; npan <= 0 skips a record)
hipError_t launch_upd_valu(const UpdArgs& g, hipStream_t stream);
// the same with one workgroup per target entry and the workgroup int8 MFMA
// product (for few entries; hipErrorInvalidValue when its LDS would exceed 160 KiB)
hipError_t launch_upd_wg(const UpdArgs& g, hipStream_t stream);
// target entries at or below which the MFMA form takes launch_upd_wg
constexpr size_t kUpdWgEntries = 1024;
hipError_t launch_upd_valu_batch(const UpdArgs* tab, int count, int nr_max, int nc_max, int nw_max, int nl_max,
                                 hipStream_t stream);

}  // namespace hl

namespace hl {
// exact update with int8-digit MFMA GEMMs
// register window of the int8 MFMA tile loop (k_upd_mfma.hip)
constexpr int kRawBufferWord3 = 0x00020000;  // gfx9 buffer descriptor word 3 (32-bit data format)
constexpr int MF_T = 16;             // output digits per accumulation block
constexpr int MF_LPB = MF_T / 4;     // limbs per block (one 16-byte slab of an entry)
constexpr int MF_PF = 8;             // operands are loaded this many steps ahead
constexpr int MF_WIN = MF_T + 2 * MF_PF;  // B window: MF_T slices in use, the rest in flight
constexpr int MF_ROT = MF_WIN / 2;   // steps per rotation of the window (a multiple of MF_PF)
static_assert(MF_ROT % MF_PF == 0, "the A ring must turn a whole number of times per rotation");
// zero slices needed at each end of the digit panels: the loads run MF_PF steps
// (2 MF_PF slices) ahead and the steps are rounded up to whole rotations
constexpr int MF_PAD_MIN = 2 * (MF_ROT + MF_PF) + 14;

struct MfmaArgs {
  UpdArgs g;
  int8_t* bdig;       // [slices][NT][16] digits of b (slice index = digit + pad)
  int8_t* udig;       // [slices][NT][16] digits of u
  int slices, pad, S, NT;
  long long* carry;   // per (tile, range, entry) carries between limb ranges
  int max_ranges;
  size_t carry_tiles; // capacity of carry in units of 1024 entries
  hl_timing_t* timing;  // host: when set, the GEMM kernel alone is timed into ms[6]
  int u_rows;           // rows of the u operand (NT for the Schur update, k for X)
};
hipError_t launch_upd_mfma(const MfmaArgs& m, hipStream_t stream);

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


// Output-limb ranges of one MFMA launch: output block boundaries tb[0..n]
// (a block is 16 digits = 4 limbs).
constexpr int MF_MAX_RANGES = 64;
struct RangeTab {
  int n;                        // ranges
  int tb[MF_MAX_RANGES + 1];    // block boundaries, tb[0] = 0, tb[n] = nw / 4
};
RangeTab make_ranges(int nl, int S, int ntiles, int max_ranges, size_t max_items);
RangeTab split_ranges(int nl, int S, int n);
// the same for ntb output blocks of a product of S-digit operands, with units
// work items per range (tiles x products)
RangeTab make_ranges_ntb(int ntb, int S, long units, int max_ranges, size_t max_items);
RangeTab split_ranges_ntb(int ntb, int S, int n);
double block_work(int tb, int S);  // digit pairs multiplied for output block tb
constexpr int MF_BLOCK_DIGITS = 16;

// Karatsuba form of the Schur update, one to three levels.  With X = 256^h,
// h = S/2, each factor splits into its balanced digits below and above h:
// b = b_lo + X b_hi, and b_mid = b_lo + b_hi is recoded into h + 1 balanced
// digits.  Then
//   sum_i b_ri u_ci = LL + X (MM - LL - HH) + X^2 HH,
// LL = sum_i b_lo u_lo, HH = sum_i b_hi u_hi, MM = sum_i b_mid u_mid: three
// digit-sum GEMMs of (h + 1)-digit operands, 3/4 of the int8 multiply-adds of
// the S-digit product.  Level l + 1 splits every level-l operand again at digit
// S/2^(l+1): 3^L GEMMs of (S/2^L + L)-digit operands after L levels, (3/4)^L of
// the multiply-adds.  The exact sums of every product are stored per entry;
// then one pass per entry subtracts sum_p c_p(Y) P_p, Y = 256^(S/2^L), c_p the
// product of the levels' polynomials (1 - z), (z^2 - z), z (children lo, hi,
// mid) at z = Y^(2^(L-l)), from the trailing matrix with exact carries.
struct KaraArgs {
  MfmaArgs m;          // target, pad, NT, carry slots (np x tiles x ranges), timing; bdig/udig unused;
                       // S here is the digit count of the split strings, a multiple of 16 x 2^L at
                       // least 4 nl (the digits above 4 nl are zero)
  int levels;          // L = 1 .. 3; np = 3^L products
  // level-l digit panels, l = 1 .. L: 3^l of b, then 3^l of u, pan_stride[l]
  // bytes apart, pan_slices[l] = S/2^l + l + 2 pad slices each; panel 3 q + c of
  // a side is child c (lo, hi, mid) of its level-(l-1) panel q
  int8_t* pan[KA_MAX_LEVELS + 1];
  size_t pan_stride[KA_MAX_LEVELS + 1];
  int pan_slices[KA_MAX_LEVELS + 1];
  int Sk;              // digits per operand of a product (kara_leaf_digits)
  int kslices;         // Sk + 2 pad
  u32* prod;           // products: [prod_tiles][np] tiles of nwp limbs per entry (a launch tile's np together)
  int nwp;             // limbs per product entry: 4 x output blocks of a (2 Sk - 1)-digit product
  size_t prod_tiles;   // tiles per product
};
hipError_t launch_upd_kara(const KaraArgs& k, hipStream_t stream);
// its pieces: the digit panels of every level before the GEMMs, and after them
// the range carries and the combination into the trailing matrix
hipError_t launch_kara_prep(const KaraArgs& k, hipStream_t stream);
hipError_t launch_kara_finish(const KaraArgs& k, const RangeTab& rt, int C_lo, int ntiles, hipStream_t stream);
// the digit-sum GEMMs alone (k_upd_mfma.hip), 8 x per_xcd work items
hipError_t launch_kara_gemm(const KaraArgs& k, const RangeTab& rt, int C_lo, int ntiles, int per_xcd,
                            hipStream_t stream);
__host__ __device__ __forceinline__ int kara_leaf_digits(int S, int levels) { return (S >> levels) + levels; }
__host__ __device__ __forceinline__ int kara_nwp(int S, int levels) {
  return 4 * ((2 * kara_leaf_digits(S, levels) - 1 + 15) / 16);
}
__host__ __device__ __forceinline__ constexpr int kara_products(int levels) {
  return levels <= 0 ? 1 : 3 * kara_products(levels - 1);
}
// digits beyond S/2^l of level-l panel q (base-3 path, most significant digit
// first): lo children have none, hi children their parent's, mid children one more
__host__ __device__ __forceinline__ int kara_extra(int q, int l) {
  int e = 0, div = 1;
  for (int j = 1; j < l; ++j) div *= 3;
  for (int j = 0; j < l; ++j) {
    const int c = (q / div) % 3;
    e = c == 0 ? 0 : (c == 1 ? e : e + 1);
    div /= 3;
  }
  return e;
}
// digits of the operands of product p at the leaf level L (its own length; the
// panel holds Sk = S/2^L + L, the rest zero)
__host__ __device__ __forceinline__ int kara_prod_digits(int S, int L, int p) { return (S >> L) + kara_extra(p, L); }

// Batched form: one entry per instance and step, work items (entry, tile index
// of the entry's launch, range) in 8 per-XCD queues of per_xcd items (x < 0:
// none); heads: 8 counters of device memory.
struct MfmaEntry {
  MfmaArgs m;
  RangeTab rt;
  int C_lo;
  int ntiles;
  // null: the sums are subtracted from the target (m.g); else the exact sums of
  // launch tile lt are stored at store + lt * store_ts, tiles of store_nw limbs
  // per entry (a Karatsuba product of the digit panels m.bdig, m.udig)
  u32* store;
  int store_nw;
  size_t store_ts;
};
struct RecodeArgs {
  const u32* src;
  size_t lds;
  int npan, NT, nrows, nl, pad;
  int8_t* dst;
};
// rows_limbs_max: the largest NT x nl of the records
hipError_t launch_recode_batch(const RecodeArgs* tab, int count, int rows_limbs_max, hipStream_t stream);
hipError_t launch_upd_mfma_batch(const MfmaEntry* tab, const int4* items, int per_xcd, unsigned* heads,
                                 hipStream_t stream);
hipError_t launch_carry_fix_batch(const MfmaEntry* tab, int count, int nrow_max, int ncol_max, hipStream_t stream);
}  // namespace hl

namespace hl {
hipError_t launch_trsm_row(const u32* ACC, const Dims& dm, int r, const i32* s, const i32* h, u32* X,
                           DevStatus* st, hipStream_t stream);
struct TrsmRowArgs {
  const u32* ACC;
  Dims dm;
  int r;
  const i32* s;
  const i32* h;
  u32* X;
  DevStatus* st;
};
hipError_t launch_trsm_row_batch(const TrsmRowArgs* tab, int count, int k_max, int nl_max, hipStream_t stream);
hipError_t launch_block(const u32* X, const Dims& dm, const u32* omega, int ostride, const i32* s,
                        u32* part, int ns, int nchunks, int rows_per_chunk, u32* msum, int nm, u32* blk,
                        i64* blk_exp, DevStatus* st, hipStream_t stream);
hipError_t launch_block_sums(const Dims& dm, const i32* s, const u32* part, int ns, int nchunks, u32* msum, int nm,
                             u32* blk, i64* blk_exp, DevStatus* st, hipStream_t stream);
// MFMA form of the block sums (see k_block_y)
hipError_t launch_block_y(const u32* X, const Dims& dm, const u32* omega, int ostride, u32* Y, int ny,
                          DevStatus* st, hipStream_t stream);
hipError_t launch_block_gather(const u32* M, const u32* M2, int nm, const Dims& dm, u32* part, int ns, DevStatus* st,
                               hipStream_t stream);
hipError_t launch_eig(const u32* blk, const Dims& dm, void* eig_ws, DevStatus* st, hipStream_t stream);
struct EigArgs {
  const u32* blk;
  int k, nl, P, NWM;
  int* hdr;
  u32* mant;
  size_t nums_per;
  int* flags;
  DevStatus* st;
  int maxit;  // iteration limit of each block's eigen-step
};
EigArgs eig_args(const u32* blk, const Dims& dm, void* eig_ws, DevStatus* st);
// the same eigen-step driven from the host, one workgroup per product (synchronises)
// aux: an optional second stream for the (k-1) x (k-1) block (nullptr: one stream)
// maxit: iteration limit per block (0: the default, 400); ENOCONV beyond it
hipError_t launch_eig_host(const u32* blk, const Dims& dm, void* eig_ws, DevStatus* st, hipStream_t stream,
                           hipStream_t aux = nullptr, int maxit = 0);
hipError_t launch_eig_batch(const EigArgs* tab, int count, int nl_max, hipStream_t stream);
void eig_result_refs(const Dims& dm, void* eig_ws, int which, int** hdr_out, u32** mant_out);
void eig_vector_refs(const Dims& dm, void* eig_ws, int** hdr_out, u32** mant_out);
// the next eigenvalues by deflation (after launch_eig_host; synchronises)
hipError_t launch_eig_next(const u32* blk, const Dims& dm, void* eig_ws, int count, DevStatus* st,
                           hipStream_t stream);
void eig_next_refs(const Dims& dm, void* eig_ws, int mat, bool diff, int** hdr_out, u32** mant_out);
int* eig_iter_ref(void* eig_ws, int mat);
}  // namespace hl

namespace hl {
// adjoint of lambda_1 (first-order perturbation of the block's largest eigenvalue)
hipError_t launch_adj_y(const int* yhdr, const u32* ymant, int NWM, const Dims& dm, const i32* s, u32* Y, u32* Yc,
                        u32* ysq, DevStatus* st, hipStream_t stream);
hipError_t launch_adj_g(const u32* X, const u32* Yc, const u32* omega, int ostride, const Dims& dm, long eG, u32* ACC,
                        DevStatus* st, hipStream_t stream);
hipError_t launch_adj_row(const u32* ACC, const Dims& dm, int i, const i32* h, u32* Z, DevStatus* st,
                          hipStream_t stream);
hipError_t launch_adj_contract(const u32* dmu, const i64* dexp, const int* dneg, int w, const Dims& dm, const i32* s,
                               i64* wprime, const u32* Z, u32* part, unsigned long long* col, u32* tot,
                               DevStatus* st, hipStream_t stream);
// MFMA form of the contraction (see k_adj_da, k_adj_part)
hipError_t launch_adj_wprime(const u32* dmu, const i64* dexp, int w, const Dims& dm, const i32* s, i64* wprime,
                             hipStream_t stream);
hipError_t launch_adj_da(const u32* dmu, const i64* dexp, const int* dneg, int w, const Dims& dm, const i32* s,
                         const i64* wprime, int j0, int npan, u32* DA, int lda, DevStatus* st, hipStream_t stream);
hipError_t launch_adj_finish(const u32* R, int nr, const u32* Z, const Dims& dm, u32* part, unsigned long long* col,
                             u32* tot, DevStatus* st, hipStream_t stream);
}  // namespace hl

namespace hl {
hipError_t launch_mfma_probe(int* out, hipStream_t stream);
}  // namespace hl

namespace hl {
// Exact update A[r][c] -= sum_i b_ri u_ci with int8 MFMA GEMMs in Toeplitz form
// (narrow targets: few columns, any rank npan <= 16).  A work item is 32 rows x
// one column x TP_DIGITS output digits.
constexpr int TP_DIGITS = 512;    // output digits (128 limbs) per work item
constexpr int TP_MAX_RANGES = 64; // output ranges per entry (entries of up to 8192 limbs)
constexpr int TP_PADB = 640;      // zero digits after the S digits of each b row
constexpr int TP_PADU_LO = 576;   // zero digits before / after the reversed digits of each u
constexpr int TP_PADU_HI = 1216;
__host__ __device__ __forceinline__ int tp_bstride(int S) { return S + TP_PADB; }
__host__ __device__ __forceinline__ int tp_ustride(int S) { return TP_PADU_LO + S + TP_PADU_HI; }
__host__ __device__ __forceinline__ int tp_ranges(int nw) { return (4 * nw + TP_DIGITS - 1) / TP_DIGITS; }
struct ToepArgs {
  UpdArgs g;           // target, factors, ranges; g.nw = limbs of a target entry
  int8_t* bd;          // [npan][NT][tp_bstride(Sb)] digits of b_r, rows RB_lo*32 .. up
  int8_t* ud;          // [npan][ncols][tp_ustride(Su)] digits of u_c, reversed
  long long* carry;    // 32 carries per work item
  size_t bd_bytes, ud_bytes, carry_words;  // capacities (host checks)
  int S, NT;           // S: digits of an nl-limb factor (4 nl)
  // optional (0: the trailing-matrix defaults)
  int nlb, nlu;        // limbs of b_r and of u_c (0: g.nl)
  size_t ucs;          // u_c at Uop + il*ldu + c*ucs (0: nlu)
  int plain;           // 1: entry (r, c) at A + r*ldr + c*ldc (limbs), else tile storage
  size_t ldr, ldc;
  int add;             // 0: A -= sum b u, 1: A += sum b u, 2: A = sum b u
  // derived by the launcher
  int RB_lo, nrb, ncols, nrg, Sb, Su;
  unsigned char rg_order[TP_MAX_RANGES];  // output ranges, most steps first
};
hipError_t launch_upd_toep(const ToepArgs& a, hipStream_t stream);
// batched form: prepare each record on the host (derived fields, checks), then
// one set of launches over a device table (grid.y = record; npan <= 0 skips)
hipError_t toep_prepare(ToepArgs& a, bool* empty);
void toep_extents(const ToepArgs& a, size_t* nb, size_t* nu, size_t* items, size_t* entries);
hipError_t launch_upd_toep_batch(const ToepArgs* tab, int count, size_t nb_max, size_t nu_max, size_t items_max,
                                size_t entries_max, int nrg_max, hipStream_t stream);
}  // namespace hl
