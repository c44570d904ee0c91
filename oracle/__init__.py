"""CPU reference oracle for the LOR-Schwarz preconditioned CG solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or runs
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP library.

Everything here is plain float64 NumPy/SciPy, written for readability rather
than speed, and follows the paper (Pazner, "Efficient low-order refined
preconditioners for high-order matrix-free continuous and discontinuous
Galerkin methods"):

* ``gll``      -- Gauss-Lobatto nodes/weights and the Lagrange derivative matrix
                  (Section 3.1, the G-NI setting).
* ``mesh``     -- structured tensor-product meshes, trilinear element maps,
                  node numbering (Section 2).
* ``highorder``-- assembled high-order CG stiffness K_p and right-hand side
                  (eq. fem / eq. system), and the IP / BR2 DG operators
                  (eq. ip, eq. br2).
* ``lor``      -- the low-order refined Q1 operator on the Gauss-Lobatto
                  sub-mesh and its element-structured coarsening hierarchy
                  (Sections 3.1 and 3.3).
* ``mdf``      -- minimum-discarded-fill ordering and the ILU(0) factor it
                  produces (Section 3.4).
* ``schwarz``  -- patch V-cycles, the coarse space, the additive Schwarz
                  preconditioner (eq. as) and its DG extension (eq. dg-as).
* ``krylov``   -- preconditioned and flexible conjugate gradients.

Where the paper is silent the oracle follows one documented reading; each
function's docstring states it.
"""
