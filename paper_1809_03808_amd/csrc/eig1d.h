// Host FP64 eigen-setup of the 1D absorbing-boundary pencil (eig1d.cpp).
#pragma once

#include <complex>
#include <vector>

namespace helm {

// The face coefficient g of du/dn + g u = 0 (outward normal) for the
// first-order absorbing condition du/dn - i omega u = 0 (g = -i omega) or a
// Neumann face (g = 0).
inline std::complex<double> face_gamma(double omega, int absorbing) {
  return absorbing ? std::complex<double>(0.0, -omega) : std::complex<double>(0.0, 0.0);
}

// All eigenpairs of K v = lambda M v for the 1D matrices of eqs. (matrixK),
// (matrixM) on n nodes with mesh size h, K's corner entries 1/h + glo and
// 1/h + ghi (face coefficients g, see face_gamma).
// Eigenvectors are normalised v^T M v = 1; v0[l] = v_l(0), v1[l] = v_l(n-1),
// and, if vfull is given, (*vfull)[i n + l] = v_l(i) (n x n, row-major).  If
// lam_lo is given, lam[l] + lam_lo[l] is the eigenvalue to extended precision
// (the refinement runs in long double).  Returns a HELM_* status.
int eig1d(int n, double h, std::complex<double> glo, std::complex<double> ghi,
          std::vector<std::complex<double>>& lam, std::vector<std::complex<double>>& v0,
          std::vector<std::complex<double>>& v1, std::vector<std::complex<double>>* vfull = nullptr,
          std::vector<std::complex<double>>* lam_lo = nullptr);

}  // namespace helm
