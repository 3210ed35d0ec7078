// Host dense Hermitian eigensolver (eig.cpp).
#pragma once

#include <complex>
#include <vector>

namespace ndq {
// Eigen-decomposition of the n x n Hermitian matrix a (row-major, destroyed):
// w ascending, z column j = eigenvector j (row-major n x n).
int hermitian_eig(int n, std::vector<std::complex<double>>& a, std::vector<double>& w,
                  std::vector<std::complex<double>>& z);
}  // namespace ndq
