// Triangular solve (Algorithm 4) and the H^-1 block (eq. equ:index): filled in below.
#include "hl_kernels.hpp"
