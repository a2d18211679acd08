"""FP64 CPU oracle for the overlapping-Schwarz optical-flow solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The library and its Python binding never call it; the oracle shares
no code, tables or helpers with the HIP path.

It is a plain, slow, obviously-correct restatement of the paper's method
(Gilliocq-Hirtz & Belhachmi, "A massively parallel multi-level approach to a
domain decomposition method for the optical flow estimation with varying
illumination"):

* ``fem``      - P1 finite elements on the two-triangles-per-pixel mesh, global
                 assembly of the Euler-Lagrange system of functional (BW2)
                 with rho = 0 (Section 2.1-2.2, equations (weakform) and
                 (discret-form)); exact integration from the moment formula.
* ``schwarz``  - image decomposition with overlap and the additive Schwarz
                 iteration with Dirichlet transmission (Section 3.1-3.2,
                 equation (schwarz)), in its restricted-additive form and in the
                 paper's Dirichlet form; subdomain solves by LAPACK banded
                 Cholesky; dense global solve for tiny grids.
* ``adapt``    - residual error indicator eta_K (equation (errind)) and the
                 alpha decrease rule (Section 2.3).
* ``metrics``  - AAE and EE (Section 4).
* ``variants`` - Gaussian presmoothing of the frames (Section 1) and the
                 area/perimeter choice of the image split (Section 3.1).
* ``adjoint``  - gradients of a loss of the solution with respect to the
                 frames and alpha by the adjoint of the discrete system.
* ``clg``      - the data term smoothed by K_rho (functionals (BW) and (BW2)
                 with rho > 0) and its error indicator.

Functions whose result the paper does not fix by any printed value or closed
form are marked "parity unpinned" in their docstrings.
"""
