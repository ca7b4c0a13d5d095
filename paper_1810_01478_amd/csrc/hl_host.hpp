// Host-side constants and the workspace layout.
#pragma once
#include <stddef.h>
#include "hl_internal.hpp"

namespace hl {

constexpr int kMaxPrec = 57344;   // pivot kernel keeps ~9 (P/32 + 8) words in LDS
constexpr int kDigitPad = 64;     // zero digit slices below 0 and above S-1
constexpr int kMaxRanges = 64;    // output-limb ranges per tile in the MFMA updates
constexpr int kBlockRows = 16;    // rows per partial sum of the H^-1 block
constexpr int kKaraMinPrec = 8192;   // by default one Karatsuba level of the Schur update from this precision on
constexpr int kKara2MinPrec = 16384; // two levels from this one
constexpr int kKara3MinPrec = 32768; // three levels from this one
constexpr int kKara4MinPrec = 40960; // four levels from this one (between 32768 and 49152 bits)
// levels deeper than the default for P are offered only while their products
// fit in this many bytes (a factorisation at the default level does not carry
// the deeper levels' buffers)
constexpr size_t kKaraExtraBytes = (size_t)16 << 30;
inline int kara_auto_level(int P) {
  return P >= kKara4MinPrec ? 4 : P >= kKara3MinPrec ? 3 : P >= kKara2MinPrec ? 2 : P >= kKaraMinPrec ? 1 : 0;
}

struct Layout {
  size_t status, tiles, upanel, omega, bdig, udig, carry, blk_part, blk_sum, eig, total;
  size_t carry_tiles;  // carry slots of 1024 entries
  // adjoint: Y and Yc (k x nl each), sum Y^2 (2 nl + 2), z (NT x nl), W' (int64),
  // per-row parts (N x (4 nl + 4)), their column sums (u64) and total (4 nl + 4)
  size_t adj_y, adj_yc, adj_ysq, adj_z, adj_wp, adj_part, adj_col, adj_tot;
  // Toeplitz-form MFMA updates: b digits, reversed u digits, carries
  size_t toep_b, toep_u, toep_carry;
  size_t toep_b_bytes, toep_u_bytes, toep_carry_words;
  size_t colprod;      // column products u_r w_i: NT rows of colprod_ld limbs
  int colprod_ld;
  size_t blk_y, blk_m;  // MFMA block sums: y_rb = x_rb w_r ([k][NT][blk_ny]), M ([k][k][blk_nm])
  int blk_ny, blk_nm;
  size_t adj_da, adj_r;  // MFMA adjoint contraction: da for 16 columns ([16][N][nw]), R ([N][adj_nr])
  int adj_nr;
  int omega_stride;
  int digit_slices;
  int blk_stride;
  int blk_chunks;
  // Karatsuba form of the Schur update: the digit panels of level l = 1 .. 3
  // (2 x 3^l panels of kara_pan_slices[l] slices, kara_pan_bytes[l] apart) and
  // the products (3^L x kara_tiles tiles for the deepest L the shape allows)
  size_t kara_pan[KA_MAX_LEVELS + 1], kara_pan_bytes[KA_MAX_LEVELS + 1], kara_prod, kara_tiles;
  int kara_pan_slices[KA_MAX_LEVELS + 1];
};

hl_status fail(hl_status s, const char* fmt, ...);
hl_status make_dims(const hl_shape* sh, Dims* dm);
Layout make_layout(const Dims& dm);
size_t eig_ws_bytes(const Dims& dm);
hl_status read_lambda(const Dims& dm, void* eig_ws, int64_t bexp, uint32_t* lam_mant, uint32_t* lam_mant_km1,
                      hl_lambda_t* out);
// the eigen-step iteration limit set on a context (0: the default)
int ctx_eig_maxit(const hl_ctx* ctx);
// looks up, once per device, the device address of hl_lambda_min_noalloc's scratch
hipError_t noalloc_init(int device);
struct ToepArgs;
// Toeplitz-form update record over a workspace's digit and carry regions
ToepArgs toep_args(const UpdArgs& g, const Layout& L, char* base, const Dims& dm);

}  // namespace hl
