"""FP64 CPU oracle for the mixed-quadrature (half-range x full-range Gauss-Hermite)
lattice Boltzmann time step of Ambrus & Sofonea, "Half-range lattice Boltzmann models
for the simulation of Couette flow using the Shakhov collision term" (arXiv:1702.01335).

THIS PACKAGE IS TEST INFRASTRUCTURE. It is a plain, slow, obviously-correct restatement
of the paper's method in numpy (float64) and mpmath (quadrature tables). Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it. The
product path (the HIP library under ``paper_1702_01335_amd``) never imports, links or
calls anything here, and this package never imports the product.

Modules
-------
quadrature   Gauss rules: half-range Hermite on the x semi-axes (Sec. III), full-range
             probabilists' Hermite on y and z (Eqs. H_omega, H_ortho).
equilibrium  Hermite-projected discrete equilibrium (Eqs. phieq, fyz, Fmn_def and the
             direct-product construction of Sec. III), Shakhov factor (Eq. sdef).
solver       moments (Eq. qdef), relaxation-time laws (Secs. IV-VI), grid (App. A.2),
             WENO-5 / 2nd-order upwind fluxes (App. A.3), boundary ghosts (App. A.4),
             TVD RK3 (App. A.1), residual.
diagnostics  Sec. IV / VI observables (u_slip, u'(0), mass flow, mean T_xy, nu, Pi, T_0).
warmstart    seed populations from predicted profiles: discrete equilibrium times the
             stress and heat-flux (Shakhov-form, Eq. sdef) correction polynomial.
mlp          the warm-start network: forward, MSE loss, chain-rule gradient with the
             bfloat16 rounding points of the GPU kernels, AdamW.

Parity status of each function is given in its docstring; functions without an
independent pin say "parity unpinned".
"""
