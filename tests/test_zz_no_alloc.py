"""The allocation-free mass entry point (sdg_mass_noalloc) against sdg_mass,
called through the C ABI: bitwise equal results on two calls in a row, the
second on a smaller mesh in another context (the static scratch keeps the
first call's contents), and again after the first context's own sdg_mass."""

import ctypes

import numpy as np
import pytest

import paper_2605_16082_amd as P
import workloads as W
from paper_2605_16082_amd.slimdg import _check, _ptr

pytestmark = pytest.mark.gpu


def _mass_noalloc_abi(s, T):
    out = np.zeros(s.mesh.n_members * s.n_fields, dtype=np.float64)
    _check(s.lib.sdg_mass_noalloc(s.ctx, _ptr(T), out.ctypes.data_as(ctypes.c_void_p)))
    return out


def _mass_abi(s, T):
    out = np.zeros(s.mesh.n_members * s.n_fields, dtype=np.float64)
    _check(s.lib.sdg_mass(s.ctx, _ptr(T), out.ctypes.data_as(ctypes.c_void_p)))
    return out


def test_mass_noalloc_matches_mass_two_calls():
    big = W.zlevel_ensemble(n_members=4, n_lo=40, n_hi=60)       # several members, 5-60 layers
    small = W.tiny(n_fields=2)
    sb, _, _, xb = P.from_workload(big, P.SDG_FP64)
    ss, _, _, xs = P.from_workload(small, P.SDG_FP32_STATE_FP64_SOLVE)
    first = _mass_noalloc_abi(sb, xb)
    ref_b = _mass_abi(sb, xb)
    print("big", first, ref_b)
    assert np.array_equal(first, ref_b)
    second = _mass_noalloc_abi(ss, xs)                             # smaller input, other context
    ref_s = _mass_abi(ss, xs)
    print("small", second, ref_s)
    assert np.array_equal(second, ref_s)
    assert second.size < first.size
    again = _mass_noalloc_abi(sb, xb)
    assert np.array_equal(again, ref_b)
