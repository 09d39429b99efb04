"""CPU oracle of fast JOFC — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct FP64 implementations of what the GPU path
computes, written from the paper's definitions:

* ``oracle.structured`` — ctypes front-end of ``fjofc_oracle.c``: the
  structured Guttman transform (eq:update with the eq:modW inverse), raw
  stress (eq. stress), Algorithm 2's loop, and the out-of-sample closed
  form (Section 3).
* ``oracle.dense`` — numpy dense tier: the omnibus W, Delta, Laplacian,
  B(X) of eq:B and the Moore-Penrose pseudo-inverse (Algorithm 1), and the
  dense out-of-sample blocks of Section 3.
* ``oracle.mlp`` — FP64 reference of the warm-start network (forward,
  backward, Adam) with the GPU path's BF16 rounding points.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU path
and never imports it.
"""
