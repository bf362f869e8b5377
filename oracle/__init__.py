"""Oracle: plain FP64 CPU reference of the four-body time-dependent NLL.

TEST INFRASTRUCTURE ONLY. It is the definition the GPU library is checked
against and shares no code with it. Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it.

The arithmetic lives in ``oracle.cpp`` (C++, compiled with g++); this module is
the ctypes shim around it. Every function follows the paper's Eq. (1), Eq. (2)
and Secs. 3 and 3.1; see the header of ``oracle.cpp``. The pseudo-experiment
generator (GENBOD phase space, Philox4x32-10 random numbers, accept-reject by
Eq. (1)) is defined there too.
"""

from .orc import (  # noqa: F401
    OracleModel,
    build,
    load,
    q2,
    barrier,
    ls_two_body,
    ls_three_body,
    spin_factors,
    basis,
    rate,
    rate_integrated,
    event_terms,
    nll,
    nll_grad,
    nll_tagged,
    max_threads,
    philox,
    candidate_uniforms,
    generate,
    OracleError,
)
