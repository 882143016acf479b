"""Inverse-free sparse variational GP training iteration for MI355X (gfx950).

The compute path is the HIP library ``_lib/libifsvgp.so`` (sources in
``csrc/``, C ABI in ``include/ifsvgp.h``); ``lib`` is its ctypes binding and
``autograd`` wraps the bound and its hand-written backward as a
``torch.autograd.Function``.  ``synth`` draws the seeded synthetic workloads.
"""
from . import synth  # noqa: F401

__all__ = ["lib", "autograd", "synth", "build"]
