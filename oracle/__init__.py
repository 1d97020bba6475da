"""FP64 CPU oracle of the Trotter-Suzuki spin propagator (arXiv:1305.0036).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline leg of
the benchmark use it; the product library never imports, links or calls it.
"""
from .oracle import (  # noqa: F401
    Hamiltonian,
    build,
    energies,
    evolve,
    expect,
    grad_forward,
    selfcheck,
    step_schedule,
    substep,
    suzuki_a,
    apply_1spin,
    apply_obs,
    OBS,
)
