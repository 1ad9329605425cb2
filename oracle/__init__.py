"""FP64 CPU oracle for image-domain gridding -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct restatement of the paper's
method (van der Tol, Veenboer & Offringa, "Image Domain Gridding", A&A 2018):
the partitioning of visibilities into subgrids (§3.2), the per-subgrid direct
imaging sum (§3.3, eq. ShiftedDirectImaging; Algorithm 1), the subgrid DFT and
the adder (Algorithm 1), and the reverse chain (Algorithm 2), with the
polarised extension of §3.4.  It exists only to check the HIP implementation.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import it.  It shares no code with the HIP library: it computes every step
itself in float64 with numpy, on the same input arrays the GPU receives.

Modules:
  plan    -- subgrid partitioning (the reading of §3.2 used by both planners)
  idg     -- gridding and degridding, subgrid by subgrid
  direct  -- direct imaging / prediction (the DIE and DME of §2) at the
             subgrid lattice, used to pin the gridder
  taper   -- classical PSWF aliasing level (§4.1, Table 1 column 2)
"""
