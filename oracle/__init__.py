"""CPU oracle for the gXY HOTRG path (test infrastructure only).

Plain, slow, FP64 numpy code written from the thesis's equations. It exists
to check the GPU library: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it. It shares no code with the
HIP path and must never be used by the product path.

Parity status of each function is stated in its docstring ("pinned by" lists
the tests in ``tests/test_oracle_pins.py`` that fix it against mathematics
that is independent of this code).
"""

from .hotrg import (  # noqa: F401
    bessel_i,
    char_coeffs,
    char_coeffs_bessel,
    field_factors,
    square_factors,
    second_moment_update,
    initial_tensors,
    environments,
    sector_eigh,
    select_states,
    project,
    hotrg_run,
    run_point,
    observables_from_runs,
    RunResult,
)
