"""Plain FP64 CPU oracle for the CPR-preconditioned FGMRES Newton solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP
library and imports nothing from it.

Every function is a direct, unblocked transcription of what the paper (Liu,
Wang & Chen, "Large-scale Reservoir Simulations on IBM Blue Gene/Q") and the
method's standard definitions state, vectorised over cells only where the
order of cells cannot change the result (cells of one colour in a red-black
sweep, independent per-cell formulas).

Modules
  model   -- black-oil / oil-water residual and analytic Jacobian (Sec. 2,
             eqs. (1)-(11)), Peaceman wells, TPFA transmissibilities
  cpr     -- quasi-IMPES decoupling, aggregation multigrid on the pressure
             block, red-black block ILU(0), the two-stage CPR apply (Sec. 2.5)
  krylov  -- restarted flexible GMRES with classical Gram-Schmidt twice
  newton  -- the inexact Newton update of Algorithm 1
  nn      -- FP64 3-D convolutional U-Net forward/backward for the learned
             pressure correction (no counterpart in the paper)
"""
