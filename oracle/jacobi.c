/*
 * Cyclic Jacobi eigensolver for a dense real symmetric matrix, FP64.
 *
 * Part of the CPU oracle (test infrastructure only).  It serves two purposes:
 *   - the explicit eigenpairs of the m x m matrix H = C^T H C once HC = CH
 *     holds at convergence (Sec. 2.1, Eq. 9), and the occasional subspace
 *     rotation that diagonalizes H (Sec. 3, discussion of MP2);
 *   - a brute-force dense eigensolve of small test Hamiltonians, which pins
 *     E_G = sum of the m lowest eigenvalues (Eq. 2) independently of the
 *     iterative solver.
 *
 * Method: the classical cyclic-by-rows Jacobi method.  Each step picks the
 * pair (p, q), p < q, builds the plane rotation J(p, q, theta) that zeroes
 * a_pq of J^T A J (the 2 x 2 symmetric Schur decomposition with the smaller
 * tangent root), and accumulates V <- V J.  Sweeps repeat until the
 * off-diagonal Frobenius norm falls below tol * ||A||_F.
 *
 * Layout: A and V are n x n, row-major.  A is overwritten (its diagonal holds
 * the eigenvalues on exit).  On exit the eigenvalues are sorted ascending into
 * w[0..n-1] and column j of V is the unit eigenvector of w[j].
 * Returns the number of sweeps used, or -1 if max_sweeps was reached first.
 */
#include <math.h>
#include <stddef.h>

static double off_norm(const double *a, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i != j)
                s += a[(size_t)i * n + j] * a[(size_t)i * n + j];
    return sqrt(s);
}

static double frob_norm(const double *a, int n)
{
    double s = 0.0;
    for (size_t k = 0; k < (size_t)n * n; ++k)
        s += a[k] * a[k];
    return sqrt(s);
}

int tmo_jacobi_eigh(int n, double *a, double *w, double *v, double tol,
                    int max_sweeps)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            v[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;

    const double anorm = frob_norm(a, n);
    int sweeps = 0;
    int converged = (n < 2) || off_norm(a, n) <= tol * anorm;
    while (!converged && sweeps < max_sweeps) {
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (apq == 0.0)
                    continue;
                const double app = a[(size_t)p * n + p];
                const double aqq = a[(size_t)q * n + q];
                /* tan(theta) is the smaller root of t^2 + 2 tau t - 1 = 0 */
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0.0)
                    ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                    : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                /* A <- A J : columns p and q */
                for (int k = 0; k < n; ++k) {
                    const double akp = a[(size_t)k * n + p];
                    const double akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - s * akq;
                    a[(size_t)k * n + q] = s * akp + c * akq;
                }
                /* A <- J^T A : rows p and q */
                for (int k = 0; k < n; ++k) {
                    const double apk = a[(size_t)p * n + k];
                    const double aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - s * aqk;
                    a[(size_t)q * n + k] = s * apk + c * aqk;
                }
                a[(size_t)p * n + q] = 0.0;
                a[(size_t)q * n + p] = 0.0;
                /* V <- V J */
                for (int k = 0; k < n; ++k) {
                    const double vkp = v[(size_t)k * n + p];
                    const double vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = c * vkp - s * vkq;
                    v[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
        }
        ++sweeps;
        converged = off_norm(a, n) <= tol * anorm;
    }

    for (int i = 0; i < n; ++i)
        w[i] = a[(size_t)i * n + i];
    /* insertion sort of the eigenvalues, carrying the columns of V along */
    for (int i = 1; i < n; ++i) {
        for (int j = i; j > 0 && w[j] < w[j - 1]; --j) {
            const double tw = w[j];
            w[j] = w[j - 1];
            w[j - 1] = tw;
            for (int k = 0; k < n; ++k) {
                const double tv = v[(size_t)k * n + j];
                v[(size_t)k * n + j] = v[(size_t)k * n + j - 1];
                v[(size_t)k * n + j - 1] = tv;
            }
        }
    }
    return converged ? sweeps : -1;
}
