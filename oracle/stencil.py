"""7-point constant-coefficient stencil on a box, Dirichlet 0 (oracle; test infrastructure).

This is the Arnoldi mat-vec w_i = A q_{i-1} of Algorithm 3 (Sec. 4.1) for the
convection-diffusion systems the solver is exercised on.  The grid is
nx x ny x nz, unknowns ordered lexicographically with x fastest
(l = x + nx*(y + ny*z)); neighbours outside the box contribute zero.

    (A u)_l = c0 u_l + cxm u_{x-1} + cxp u_{x+1} + cym u_{y-1} + cyp u_{y+1}
                     + czm u_{z-1} + czp u_{z+1}
"""

import numpy as np


def apply(u, dims, coeffs, dtype=np.float64):
    """w = A u.  dims = (nx, ny, nz); coeffs = (c0, cxm, cxp, cym, cyp, czm, czp).

    ``dtype`` is the arithmetic type (float64, or float32 for the working
    precision of the multi-precision model).
    """
    nx, ny, nz = dims
    c0, cxm, cxp, cym, cyp, czm, czp = [dtype(c) for c in coeffs]
    U = np.asarray(u).astype(dtype).reshape(nz, ny, nx)
    Up = np.zeros((nz + 2, ny + 2, nx + 2), dtype=dtype)
    Up[1:-1, 1:-1, 1:-1] = U
    c = Up[1:-1, 1:-1, 1:-1]
    w = c0 * c
    w = w + cxm * Up[1:-1, 1:-1, :-2]
    w = w + cxp * Up[1:-1, 1:-1, 2:]
    w = w + cym * Up[1:-1, :-2, 1:-1]
    w = w + cyp * Up[1:-1, 2:, 1:-1]
    w = w + czm * Up[:-2, 1:-1, 1:-1]
    w = w + czp * Up[2:, 1:-1, 1:-1]
    return w.reshape(-1)
