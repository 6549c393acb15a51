"""Plain, slow CPU FP64 oracle for the moving-PML sweeping preconditioner.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package; only the tests, the smoke check and the benchmark's CPU-baseline leg
do.  The oracle shares no code with the GPU path: it takes plain NumPy arrays
(velocity, right-hand sides) that the seeded input generators produce and
computes everything else itself, in complex128, with SciPy's sparse LU and
NumPy as its only library primitives.

Modules, each citing the passage of Poulson, Engquist, Li and Ying,
"A parallel sweeping preconditioner for heterogeneous 3D Helmholtz
equations" that it follows:

* ``helmholtz`` -- the grid, the complex-stretched PML and the 7-point
  discretisation of the Helmholtz operator A and of the damped operator J
  (Sec. 1, Eq. 1.1; Sec. 1.1, block tridiagonal form and Eq. 1.5).
* ``panels``    -- panels and their auxiliary problems H_i (Sec. 1.1,
  Alg. 1.3 and Alg. 1.4).
* ``nd``        -- nested dissection of a quasi-2D panel into a supernodal
  elimination tree in postorder (Sec. 2.1, Fig. 2.1) and the update sets
  obtained by symbolic elimination.
* ``ldlt``      -- unpivoted complex-symmetric LDL^T and the per-front blocks
  D, L_F, F_BL of Sec. 2.2.
* ``sweep``     -- T_i = approximate inverse Schur complement (Alg. 1.3) and
  the sweep M^{-1} (Alg. 1.5).
* ``gmres``     -- right-preconditioned GMRES(k) in FP64 (Sec. 2.4).

Readings of points the paper leaves open (PML profile, where PML starts,
the symmetric stretched stencil, the panel layout, the nested-dissection cut
rule, the GMRES variant) are stated in each module's docstring.  The PML
profile sigma(t) = (C/eta)(t/eta)^2 is a reading: the paper only names the
amplitude C of a cited formula, so agreement with the paper's own profile is
parity unpinned; the profile's sign and absorption are pinned physically by
the outgoing 1D Green's function test.
"""
