"""Plain FP64 CPU oracle of the Flux Reconstruction right-hand side (TEST INFRASTRUCTURE).

This package is the independent reference that the GPU path is checked against.
Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product library never does, and shares no code with it.

Every function follows the paper's statement of the scheme (Sec. "Flux
Reconstruction": mapping and Jacobians, the transformed equation, the four steps
eq:disu / eq:comm_flux / second eq:disu / eq:FRfinal), with dense per-element
operator matrices (Kronecker products for hexahedra, Vandermonde-based for
tetrahedra) and no sum factorisation, blocking or fusion.  Where the paper is
silent (Riemann solver, correction function, viscous discretisation, time
integrator, entropy-filter internals) the reading used is stated in each module.

Modules
    polys      1-D Gauss--Legendre, Legendre, Lagrange and Radau (DG correction) polynomials
    tet        the paper's p=4 alpha-optimised tetrahedral points, orthonormal tet basis
    elements   dense element operator sets for hexahedra and tetrahedra
    pyramid    the p=4 pyramid: rational space, layered points, DG lifting (affine base)
    mesh       periodic face matching, flux-point pairing, left/right sides
    geometry   Jacobians and transformed metric at arbitrary reference points
    curved     order-q hexahedral maps; conservative (curl-form) and cross-product metrics
    physics    Euler flux, Rusanov and HLLC solvers, Navier--Stokes viscous flux
    fr         the FR right-hand side (Euler and Navier--Stokes, LDG)
    rk         classical RK4
    nodal_dg   weak-form nodal DG built by brute-force quadrature (a pin)
    entropy_filter  entropy-bounded modal filter with dyadic bisection
    mlp        16-64-64-1 tanh MLP: forward, analytic backward, Adam (FP64)
"""
