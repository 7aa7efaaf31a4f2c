"""Reference for the line factor's unpivoted inversions, in NumPy (FP64):
the block Schur recursion over x-lines of a box's local matrix,
S_0 = T_0, S_j = T_j - M_{j,j-1} S_{j-1}^-1 M_{j-1,j}, each S_j inverted by
scalar Gauss-Jordan without pivoting, with every pivot recorded.  The local
matrix comes from the oracle's assembly (Sec. 2, eq. pml times J, on the
box with its own layer); the Gauss-Jordan here is written for these tests
and shares nothing with the HIP kernels."""
import numpy as np


def line_blocks(M, mx, my):
    """Dense diagonal blocks T_j and coupling blocks M_{j,j+1} of the local
    matrix M (unknowns row-major: x-line j holds rows j*mx .. j*mx+mx-1)."""
    M = M.tocsr()
    T = [M[j * mx:(j + 1) * mx, j * mx:(j + 1) * mx].toarray() for j in range(my)]
    C = [M[j * mx:(j + 1) * mx, (j + 1) * mx:(j + 2) * mx].toarray() for j in range(my - 1)]
    return T, C


def gauss_jordan_unpivoted(S):
    """In-place Gauss-Jordan inverse with the diagonal as pivots, in order.
    Returns (inverse, pivots)."""
    A = np.array(S, dtype=np.complex128)
    n = A.shape[0]
    piv = np.empty(n, dtype=np.complex128)
    for k in range(n):
        p = A[k, k]
        piv[k] = p
        f = A[:, k].copy()
        f[k] = 0.0
        A[:, k] = 0.0
        A[k, k] = 1.0
        A[k, :] /= p
        A -= np.outer(f, A[k, :])
    return A, piv


def schur_recursion(M, mx, my):
    """Yields (j, S_j, G_j, pivots of S_j) along the box's x-lines."""
    T, C = line_blocks(M, mx, my)
    G = None
    for j in range(my):
        S = T[j] if j == 0 else T[j] - C[j - 1].T @ G @ C[j - 1]
        G, piv = gauss_jordan_unpivoted(S)
        yield j, S, G, piv
