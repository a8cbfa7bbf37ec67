"""Seeded synthetic inputs shared by the tests, the bench and the oracle.

Holds no rendering arithmetic: it only draws occupancy (unions of
ellipsoids), leaf coefficients, temporal bases, camera poses and raw ray
sets from seeded numpy generators. Both the FP64 oracle and the GPU path
consume what it returns.
"""
from .scenes import *  # noqa: F401,F403
