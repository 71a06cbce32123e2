"""CPU FP64 oracle for the level-set ILT hot path (DevelSet, arXiv 2303.12529).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this
package: only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may call it.  It shares no code with the HIP library; the only
common inputs come from ``paper_2303_12529_amd.inputs`` (seeded clips and
optical kernels), which holds none of the method's arithmetic.

Modules, each following the paper's statement of the step it computes:

* ``litho``    -- SOCS imaging (Sec. II-B, Hopkins / truncated SOCS sum) on a
                  pruned DFT window, its adjoint (Sec. III-A, the ILT gradient
                  equation), and two independent second routes used as pins
                  (the Hopkins/TCC-domain forward and the G-window adjoint).
* ``resist``   -- sigmoid resist, L_DSO = alpha L_ilt + beta L_pvb, dL/dI,
                  and the binary-print L2 / PVBand metrics (Sec. II-C, III-A).
* ``levelset`` -- central differences and curvature (Sec. III-A numerical
                  settings), the DSO evolution step with the CFL time step.
* ``edt``      -- exact squared Euclidean distance transform (plain C) and the
                  truncated signed distance function (TSDF equation, Alg. 1's
                  CUDA_TSDF role).
* ``solve``    -- the plain DSO loop in the paper's order.
* ``dsn``      -- the level-set branch of DevelSet-Net (Sec. III-B): a UNet
                  forward and backward, the L_0 squared error, Adam, and the
                  resampling between the 2048 grid and the network's 512 grid.

Everything floating-point is float64.  Readings of passages the paper leaves
open are listed in the design document; each function's docstring names the
passage it follows.
"""
