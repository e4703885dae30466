"""CPU FP64 oracle for MLMC with stabilized leapfrog local time-stepping.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import anything in this package; the
library's product path never does (it fails loudly when its HIP extension is
missing instead of falling back here).

The oracle is a plain, slow, deliberately unfused restatement of what the
method computes (Grote, Michel, Nobile: "Uncertainty quantification by MLMC
and local time-stepping for wave propagation"):

* ``mesh``     -- rectilinear level meshes (tensor grids split into P1
                  triangles), Dirichlet mask, coefficient blocks, fine-element
                  flags, projector P (Sec. 3.3), lumped mass, QoI weights.
* ``trimesh``  -- levels given as triangulations (nodes, counter-clockwise
                  triangles, Dirichlet nodes, element blocks and fine flags,
                  per-node QoI weights) with the same P1 operators.
* ``fem``      -- general P1 assembly of K(kappa) and the lumped M
                  (Sec. 3.1, mass-lumped Galerkin system).
* ``rng``      -- Philox4x64-10 samples via numpy's independent Philox,
                  Box-Muller normals, per-sample step counts.
* ``cheby``    -- the stabilized Chebyshev constants delta, omega, beta_k,
                  beta_{k+1/2} (Sec. 3.3), in exact rational arithmetic.
* ``lts``      -- Algorithm 2 (stabilized LF-LTS), literally, on all DOFs;
                  plain leapfrog; discrete energy.
* ``mlmc``     -- QoI, coupled differences, two-pass moments, optimal N_l,
                  bias estimate, Algorithm 1 (Sec. 2.2).
* ``adjoint``  -- discrete adjoint of the LF-LTS recurrence (dQ/d log c).
* ``mlts``     -- multi-level LTS (Sec. 3.5, closing remark): Algorithm 2
                  nested once per tier of element sizes, each tier with its
                  own ratio p_j (a reading; the paper names the method only).
* ``oned``     -- the one-dimensional workloads of Sec. 4.1 / 4.2 (Neumann
                  data, random wave speed by a Karhunen-Loeve sum or a random
                  jump) with the V = L^2(D)-valued QoI and its Algorithm 1.

It shares no code with the HIP path and imports nothing from it.
"""
