"""CPU oracle for RQC amplitudes — TEST INFRASTRUCTURE, not part of the product.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import or run anything in this package.  It shares no code with the HIP library: it reads
the same circuits (``rqc_inputs``) and nothing else.

Engines (FP64 throughout):
  E1  ``statevector``  state-vector simulation, and its adjoint gradient;
  E2  ``tn``           time-collapsed tensor network contracted pairwise, with explicit
                       slicing over cut bonds (per-path and partial-path amplitudes);
  E3  ``tn.linear_xeb_grad`` gradient of linear cross-entropy by autograd through E2.
``slices`` draws the seeded fraction of paths; ``metrics`` holds the error measures;
``sampling`` is the fast frugal rejection sampler over open-qubit batches and its error
estimate; ``gf2`` gives exact per-path amplitudes of CZ-only circuits at any size (exponential
sums of quadratic forms over GF(2)).
Every function is pinned by a test under ``tests/`` against something other than itself
(closed forms, special cases, the other engine, finite differences, the paper's numbers).
"""
from . import gates, gf2, metrics, sampling, slices, statevector, tn  # noqa: F401
