/*
 * rbicg_hostla.h -- host FP64 dense linear algebra used at the cycle ends of
 * recycling BiCG (librbicg.so).  Exported so that it can be checked on a CPU.
 *
 * Matrices are complex, column-major, interleaved (re, im) doubles: element
 * (i, j) of an m x n matrix sits at 2*(i + j*m).  All arrays are host memory
 * owned by the caller.  Return value: 0 on success, -1 on bad arguments or a
 * failed factorization (message in rbicg_last_error()).
 */
#ifndef RBICG_HOSTLA_H
#define RBICG_HOSTLA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Generalized eigenproblem P w = lambda Q w (Q = NULL: standard problem), the
 * form of eq. finalGenEigValue (Sec. 4.1) and of the first-cycle problem
 * T w = lambda w (Sec. 4.2), by the QZ algorithm of Moler and Stewart on the
 * pencil itself (the real double-shift variant when P and Q are real, the
 * complex single-shift variant otherwise); Q may be singular (infinite
 * eigenvalues are returned as inf).  Outputs (any may be NULL):
 *   lam[2m]    eigenvalues
 *   W[2m*m]    right eigenvectors (unit 2-norm columns)
 *   Wl[2m*m]   left eigenvectors y: y^H P = lambda y^H Q (unit 2-norm),
 *              i.e. the eigenvectors of the conjugate-transposed pencil. */
int rbicg_host_eig(int32_t m, const double *P, const double *Q, double *lam, double *W,
                   double *Wl);

/* Select eigenvectors for the k eigenvalues closest to the origin (Sec. 4.1),
 * ordered by (|lambda|, Re, Im); infinite/NaN values are skipped.  For a real
 * problem (real_problem = 1) a conjugate pair contributes the two real vectors
 * [Re w, Im w] and a real eigenvalue the real vector w (phase removed); a pair
 * that does not fit in k is dropped.  Wsel, Wlsel: m x k outputs; returns the
 * number of selected columns (>= 0), or -1. */
int rbicg_host_select(int32_t m, const double *lam, const double *W, const double *Wl,
                      int32_t k, int32_t real_problem, double *Wsel, double *Wlsel);

/* rbicg_host_eig followed by rbicg_host_select, computing eigenvectors only
 * for the selected eigenvalues (the cycle-end path).  Wsel, Wlsel: m x k
 * outputs.  Returns the number of selected columns (>= 0), or -1. */
int rbicg_host_eig_select(int32_t m, const double *P, const double *Q, int32_t k,
                          int32_t real_problem, double *Wsel, double *Wlsel);

/* Thin SVD A = U diag(s) V^H of an m x n matrix (m >= n) by one-sided Jacobi;
 * singular values descending.  U: m x n, s: n reals, V: n x n. */
int rbicg_host_svd(int32_t m, int32_t n, const double *A, double *U, double *s, double *V);

/* Hermitian eigendecomposition A = V diag(w) V^H (cyclic Jacobi), ascending. */
int rbicg_host_heig(int32_t m, const double *A, double *w, double *V);

/* Biorthogonalization step of Sec. 4.3 from Gram matrices of C = A U and
 * C~ = A^H U~ (k columns each): Gcc = C^H C, Gtt = C~^H C~, Gtc = C~^H C.
 * Orthonormal bases Q = C L, Q~ = C~ L~ come from the Hermitian eigen-
 * decompositions of Gcc and Gtt (directions with eigenvalue below
 * 1e-13 * max are dropped); Q~^H Q = M Sigma N^H; the p cosines sigma_i >= tol
 * are kept and TU = L N_p Sigma_p^{-1/2}, TUt = L~ M_p Sigma_p^{-1/2} (k x p,
 * column-major, leading dimension k) make U TU, U~ TUt a biorthogonal pair
 * (C~^H C = I_p).  Returns p (>= 0) or -1. */
int rbicg_host_biorth(int32_t k, const double *Gcc, const double *Gtt, const double *Gtc,
                      double tol, double *TU, double *TUt);

/* ILUT(tau, p) of the split preconditioning of Sec. 6 (the factorization the
 * library's rbicg_ilut_create uses), by row-wise elimination without
 * pivoting.  The n x n matrix is CSR (rowptr[n+1], colind, values interleaved
 * complex: real matrices carry zero imaginary parts).  Drop rules, scaled as
 * MATLAB's drop tolerance: when row i's elimination reaches column k < i the
 * entry w_k (before division by the pivot u_kk) is dropped if
 * |w_k| < tau ||A(:,k)||_2, and a dropped entry updates nothing; after the
 * elimination an entry w_j, j > i, is dropped if |w_j| < tau ||A(:,j)||_2; the
 * diagonal is kept; p >= 0 keeps at most p off-diagonal entries per row in
 * each factor (largest modulus first, ties by column), p < 0 no limit.
 * permtol > 0 selects ILUTP, the column-pivoting variant (Sec. 6.2): after
 * row i's elimination and dropping (the entry of the column at position i is
 * never dropped), the largest remaining entry (ties: the smallest position)
 * becomes the pivot when its modulus times permtol exceeds that of the
 * position-i column, and the two columns swap positions; the factors then
 * satisfy A Q = L U + E with (A Q)(:, j) = A(:, perm[j]) and are given in
 * positions.  permtol = 0: ILUT, perm the identity.
 * Outputs: nnz[0] = entries of L (strictly lower, unit diagonal implied),
 * nnz[1] = entries of U (with the diagonal); with Lrp/Lci/Lv (n+1, nnz[0],
 * 2*nnz[0]) and Urp/Uci/Uv non-NULL the factors in CSR, columns ascending
 * (call once with them NULL for the sizes); perm (n entries) when non-NULL.
 * -1 on bad arguments or a zero pivot. */
int rbicg_host_ilut(int32_t n, const int32_t *rowptr, const int32_t *colind,
                    const double *values, double tau, int32_t p, double permtol, int64_t *nnz,
                    int32_t *Lrp, int32_t *Lci, double *Lv, int32_t *Urp, int32_t *Uci,
                    double *Uv, int32_t *perm);

/* Level schedule of a triangular solve with the CSR matrix T (lower = 1: row
 * i depends on its columns j < i, else on j > i; other entries are ignored):
 * level(i) = 1 + the largest level of the rows it depends on (0 if none).
 * order lists the rows level by level (ascending inside a level), each level
 * padded with -1 to a multiple of pad; *len its length (order NULL: length
 * only).  Returns the number of levels, or -1. */
int rbicg_host_levels(int32_t n, const int32_t *rowptr, const int32_t *colind, int32_t lower,
                      int32_t pad, int32_t *order, int64_t *len);

#ifdef __cplusplus
}
#endif
#endif /* RBICG_HOSTLA_H */
