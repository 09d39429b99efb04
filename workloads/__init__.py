"""Seeded synthetic workloads for fast JOFC.

This package only draws random numbers and builds input dissimilarities
(Euclidean distances of latent-model views).  It holds none of the
method's arithmetic, so both the CPU oracle (tests) and the HIP path
(library, bench) can take their inputs from it without sharing code.
"""
from .generators import *  # noqa: F401,F403
