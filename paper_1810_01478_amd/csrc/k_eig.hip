// Eigen-step (filled in below).
#include "hl_kernels.hpp"
#include "hl_host.hpp"

namespace hl {
size_t eig_ws_bytes(const Dims& dm) { return (size_t)64 * 1024 + (size_t)dm.k * dm.k * (dm.nl + 8) * 4 * 8; }
}  // namespace hl
