// Host ILUT factorization and level schedules of triangular factors, for the
// split preconditioning of Sec. 6 (the experiments precondition every system
// with an ILUT-type incomplete LU factorization).
#pragma once
#include <complex>
#include <string>
#include <vector>

namespace ilut {

using cplx = std::complex<double>;

// CSR with complex values (real matrices have zero imaginary parts).
struct Csr {
  int n = 0;
  std::vector<int> rp, ci;
  std::vector<cplx> v;
};

// ILUT(tau, p) by row-wise elimination without pivoting.  Drop rules, scaled
// as MATLAB's drop tolerance: when row i's elimination reaches column k < i,
// the entry w_k (before division by the pivot u_kk) is dropped if
// |w_k| < tau ||A(:,k)||_2 and then updates nothing; after the elimination an
// entry w_j, j > i, is dropped if |w_j| < tau ||A(:,j)||_2; the diagonal is
// kept.  p >= 0 keeps at most p off-diagonal entries per row in each factor
// (largest modulus first, ties by column); p < 0: no limit.
// L: the strictly lower part (unit diagonal implied); U: upper with diagonal.
// Returns 0, or -1 with msg set on a zero pivot.
int factor(const Csr &A, double tau, int p, Csr &L, Csr &U, std::string &msg);

// ILUTP(tau, p, permtol): ILUT with column pivoting.  Positions are tracked
// as perm (position -> column of A, initially the identity); row i's lower
// part is the columns already pivotal for rows 0..i-1, eliminated in that
// order with ILUT's rule; the remaining entries are dropped by ILUT's rule
// except that of column perm[i]; the largest kept remaining entry (ties: the
// smallest position) becomes the pivot when its modulus times permtol exceeds
// that of column perm[i], and the two columns swap positions; then at most p
// off-pivot entries per part (largest modulus, ties by position).  On return
// A Q = L U + E with (A Q)(:, j) = A(:, perm[j]); L and U in positions.
// permtol = 0 never pivots.  Returns 0, or -1 with msg set on a zero pivot.
int factor_pivoted(const Csr &A, double tau, int p, double permtol, Csr &L, Csr &U,
                   std::vector<int> &perm, std::string &msg);

// Conjugate transpose.
Csr conj_transpose(const Csr &T);

// Level schedule of a triangular solve with T (lower: rows depend on smaller
// columns, else on larger): level[i] = 1 + max level of the rows it depends
// on.  order lists the rows level by level (ascending row index inside a
// level), each level padded with -1 to a multiple of pad.  Returns the
// number of levels.
int levels(const Csr &T, bool lower, int pad, std::vector<int> &order);

}  // namespace ilut
