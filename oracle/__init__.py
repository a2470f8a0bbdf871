"""Plain FP64 CPU oracle of the DG elasticity / thermal-noise method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP path: it builds its own mesh,
geometry and operator from the problem description, with dense NumPy
arithmetic written to be read against the paper:

* ``lgl``       Legendre-Gauss-Lobatto nodes, weights, differentiation
                (Sec. 2.2.1, basis of eqs. field_expansion / lagrprod)
* ``mesh``      layered cylinder of the domain decomposition (Sec. 2.2.1) and a
                layered box; faces matched by node coordinates
* ``geometry``  Jacobian, inverse, determinant, normals, surface Jacobian
                (Sec. 2.2.1, eqs. massmat / stiffmat / liftop)
* ``material``  constitutive tensors (eqs. constrel_iso, constrel_cryst)
* ``dg``        auxiliary strain, DG residual in weak and in strong form,
                generalized internal-penalty flux with averaged moduli
                (Sec. 2.2.2 - 2.2.4, eqs. dg_residuals, numflux, penalty, bc),
                load vector, energies
* ``solve``     dense and conjugate-gradient solves (Sec. 2.3)
* ``indicator`` face-jump indicator of adaptive refinement (the jump the
                penalty of eq. penalty acts on; Sec. 4)
* ``physics``   Levin noise formula and closed forms (Sec. 2.1)
* ``slab``      semi-analytic layered-slab energies per Fourier mode, used only
                to pin the physics

Parity status of each function is stated in its module header.
"""
