// Host evaluation of the envelope kernels for a constant equation of state w
// (see sigw_eos.cpp): used to build the separable tables of Sec. V for that
// background.
#pragma once

namespace sigw {

// I_s^w and I_c^w at the pairs (c[i], c[j]) with pairs[i n + j] != 0 (a
// symmetric mask); both results are written symmetrically into the n x n
// row-major matrices Is and Ic (other entries untouched).  0 < w < 1, c > 0.
// Throws std::invalid_argument / std::domain_error on bad input.
void eos_kernel_matrices(double w, const double* c, int n, const unsigned char* pairs, double* Is, double* Ic);

}  // namespace sigw
