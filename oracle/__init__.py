"""FP64 CPU oracle for the implicit ADI wave solver -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import it.  It shares no code with the HIP library.

Parity status of each function (what pins it; see tests/test_oracle_pins.py):
  thomas, tridiag_batched  -- dense LU on random diagonally dominant systems.
  step_parts, run          -- dense Kronecker operators (factored form) on tiny
                              heterogeneous grids; the unfactored eq. (CN1)
                              solved densely (one-step gap shrinks like dt^6);
                              the discrete standing-wave closed form; the
                              continuous closed form; second-order convergence;
                              the discrete energy invariant; x<->y symmetry.
  start                    -- PAPER mode: eq. (CN2) verbatim; GHOST mode: the
                              discrete standing-wave closed form from step 0.
  adjoint                  -- central finite differences of the forward loss on
                              random cells; the source-to-trace dot-product
                              identity <F f, d> = <f, F^T d>.
  step_tdc                 -- eq. (CN1) with a time-dependent coefficient: the
                              unfactored eq. (CN1) with c^{k+1}, c^{k-1} solved
                              densely (gap shrinks like dt^6); the discrete
                              closed form of a mode under a spatially constant
                              kappa(t); second-order convergence to a
                              manufactured solution with kappa(t, x, y); equal
                              to step_parts for a constant coefficient.
  step_split               -- the split as printed (eqs. (fr1)-(fr2)) and Listing
                              1's line systems: each sub-step against its printed
                              equation solved densely with Kronecker operators and
                              per-node kappa; the scalar recurrence of a grid mode
                              over many steps; the phase speed of the printed
                              split, sqrt(2) times the continuous one.
"""
from .oracle import (build, lib, max_threads, thomas, tridiag_batched, step_parts, run,
                     start, initial_levels, run_problem, adjoint, step_tdc, step_split)

__all__ = ["build", "lib", "max_threads", "thomas", "tridiag_batched", "step_parts", "run",
           "start", "initial_levels", "run_problem", "adjoint", "step_tdc", "step_split"]
