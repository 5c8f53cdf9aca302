"""Seeded synthetic inputs (meshes, permittivity, acquisition, regulariser).

Shared by the GPU library's tests and benchmark and by the oracle's tests.  It holds
no arithmetic of the method itself: meshes, classification, random numbers, wavelets.
"""
from . import acquisition, body, configs, mesh, regularizer  # noqa: F401
