"""D2Q9 lattice and the MRT moment basis.

Test infrastructure only (see oracle/__init__.py).

Follows Sec. 2 of the paper: the D2Q9 velocity set (the equation after
Eq. lbm), the equilibrium weights w_i (text after
Eq. EquilibriumDistribution), the interaction-force weights W_i = 1/3
(|c|^2 = 1) and 1/12 (|c|^2 = 2) (text after Eq. shanchen) and the
Lallemand-Luo moment matrix M printed after Eq. collisionMRT.

Parity: pinned by tests/test_oracle_lattice.py (orthogonality of the rows
of M, M^-1 M = I, moments of the equilibrium against the weight form of
Eq. EquilibriumDistribution, isotropy sums of the weights).
"""
import numpy as np

# velocity set, index i = 0..8 in the paper's order
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.int64)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.int64)

# equilibrium weights w_i
W_EQ = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])

# interaction-force weights w(|c_i|^2): 1/3 for |c|^2 = 1, 1/12 for |c|^2 = 2
W_INT = np.array([0.0, 1 / 3, 1 / 3, 1 / 3, 1 / 3, 1 / 12, 1 / 12, 1 / 12, 1 / 12])

# index of the opposite velocity
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6], dtype=np.int64)

# Lallemand-Luo moment matrix, rows: rho, e, zeta, j_x, q_x, j_y, q_y, p_xx, p_xy
M = np.array(
    [
        [1, 1, 1, 1, 1, 1, 1, 1, 1],
        [-4, -1, -1, -1, -1, 2, 2, 2, 2],
        [4, -2, -2, -2, -2, 1, 1, 1, 1],
        [0, 1, 0, -1, 0, 1, -1, -1, 1],
        [0, -2, 0, 2, 0, 1, -1, -1, 1],
        [0, 0, 1, 0, -1, 1, 1, -1, -1],
        [0, 0, -2, 0, 2, 1, 1, -1, -1],
        [0, 1, -1, 1, -1, 0, 0, 0, 0],
        [0, 0, 0, 0, 0, 1, -1, 1, -1],
    ],
    dtype=np.float64,
)

# inverse by a library solve (a primitive); the tests check it against the
# orthogonality of the rows of M
M_INV = np.linalg.inv(M)

CS2 = 1.0 / 3.0  # lattice sound speed squared
