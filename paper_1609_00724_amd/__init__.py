"""MI355X (gfx950) field-line tracer for squashing-factor (Q), field-line-length
and FLEDGE maps -- the hot path of QSL Squasher (Tassev & Savcheva 2017,
arXiv:1609.00724).

This package is a thin ctypes binding of ``libqsq.so``, whose C-ABI is
declared in ``include/qsq.h``.  PyTorch provides device memory and streams
only; every step of the path runs in the library's HIP kernels.  Importing the
package fails if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

__all__ = ["lib", "LIB_PATH", "Field", "field_init", "trace", "TracePlan", "trace_batch", "TraceBatchPlan", "fledge",
           "hilbert2_d2xy", "hilbert2_xy2d", "hilbert3_d2xyz", "hilbert3_xyz2d", "qmap", "QMapPlan",
           "MapSpec", "VolumeSpec", "QsqError"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsq.so")

# torch first: its HIP runtime (same SONAME as the system one) is then the one
# process-wide runtime that both torch and libqsq use
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python {os.path.join(_HERE, 'build.py')}` "
                      "(or __graft_entry__.build()) first")

from . import _abi  # noqa: E402
from ._abi import lib, QsqError  # noqa: E402
from .api import (Field, field_init, trace, TracePlan, trace_batch, TraceBatchPlan, fledge,  # noqa: E402
                  hilbert2_d2xy,
                  hilbert2_xy2d, hilbert3_d2xyz, hilbert3_xyz2d, qmap, QMapPlan, MapSpec, VolumeSpec)
