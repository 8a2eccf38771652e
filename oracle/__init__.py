"""CPU oracle of the hybrid DG/FV right-hand side.

TEST INFRASTRUCTURE ONLY.  A plain, slow, float64 reference written from the
paper (arXiv 2502.19342, Sections 2 and 3).  It shares no code with the HIP
library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it; the product path never does.

Modules:
    ops1d      LGL nodes/weights, D, V_Leg, degree and DG<->FV maps
    geometry   trilinear elements, curl-form metric terms, Jacobian
    physics    EOS, Euler fluxes, two-point fluxes, Riemann solvers
    rhs        the hybrid DG/FV right-hand side R(u; alpha)
    indicator  modal decay indicator and blending ramp
    lsrk       five-stage fourth-order 2N Runge-Kutta and the CFL time step
    problem    assembly of a workload into oracle objects
    limiter    positivity-preserving limiter of Zhang and Shu
    native_fv  FV-stored elements: minmod-reconstructed sub-cell means, switching
    p_adapt    degree decision from I(rho) and the state maps between degrees
    viscous    viscous multi-species fluxes and BR1 lifting
"""
