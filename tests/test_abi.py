"""The C ABI without a GPU: the library loads, exports every declared entry
point, agrees with the input layout, and rejects invalid arguments on the
host before any device call.
"""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2512_23183_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sv.h")
LIB = os.path.join(ROOT, "paper_2512_23183_amd", "libsv.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(sv_\w+)\(", text, re.M)))


@pytest.fixture(scope="module")
def sv():
    if not os.path.exists(LIB):
        pytest.fail("libsv.so is not built (run __graft_entry__.build())")
    from paper_2512_23183_amd import sv as svmod
    return svmod


def test_every_declared_symbol_is_exported(sv):
    names = _declared()
    assert len(names) >= 30
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (sv_\w+)$", out, re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = sv.lib()
    for n in names:
        assert getattr(L, n) is not None


def test_gate_kind_numbers_match_header():
    text = open(HEADER).read()
    enum = dict((k, int(v)) for k, v in re.findall(r"SV_(\w+) = (\d+)", text))
    for kind, name in I.KIND_NAMES.items():
        assert enum[name] == kind, name
    assert enum["NUM_GATE_KINDS"] == len(I.KIND_NAMES)


def test_gate_record_layout():
    # sv_gate: int32 kind, q[3], param_idx[3], mat_idx, double angle[3] = 56 B
    class G(ctypes.Structure):
        _fields_ = [("kind", ctypes.c_int32), ("q", ctypes.c_int32 * 3),
                    ("param_idx", ctypes.c_int32 * 3), ("mat_idx", ctypes.c_int32),
                    ("angle", ctypes.c_double * 3)]
    assert ctypes.sizeof(G) == I.GATE_DTYPE.itemsize == 56
    for name in ("kind", "q", "param_idx", "mat_idx", "angle"):
        assert getattr(G, name).offset == I.GATE_DTYPE.fields[name][1]


def test_version(sv):
    assert "gfx950" in sv.version()


def _circ_with(mod):
    c = I.hea_circuit(3, 1)
    g = c.gates.copy()
    mod(g)
    return I.Circuit(c.n, g, c.mats, c.n_params)


@pytest.mark.parametrize("case", [
    "qubit_range", "dup_qubit", "bad_kind", "pidx_range", "pidx_wrong_slot",
    "nan_angle", "mat_idx"])
def test_invalid_circuits_rejected(sv, case):
    params = I.uniform_params(6, 0)
    def mod(g):
        if case == "qubit_range":
            g[0]["q"][0] = 3
        elif case == "dup_qubit":
            g[-1]["q"][1] = g[-1]["q"][0]
        elif case == "bad_kind":
            g[0]["kind"] = 99
        elif case == "pidx_range":
            g[0]["param_idx"][0] = 6
        elif case == "pidx_wrong_slot":
            g[0]["param_idx"][1] = 0
        elif case == "nan_angle":
            g[0]["angle"][0] = math.nan
        elif case == "mat_idx":
            g[0]["kind"] = I.MAT1
            g[0]["param_idx"][0] = -1
            g[0]["mat_idx"] = 0
    c = _circ_with(mod)
    with pytest.raises(sv.SvError) as e:
        sv.check_circuit(c, params)
    assert e.value.name == "SV_EINVAL"


def test_param_vector_checks(sv):
    c = I.hea_circuit(3, 1)
    sv.check_circuit(c, I.uniform_params(6, 0))
    for bad in (np.zeros(5), np.zeros(7), np.array([0, 0, math.inf, 0, 0, 0.0]),
                np.array([0, 0, 0, 0, 0, math.nan])):
        with pytest.raises(sv.SvError) as e:
            sv.check_circuit(c, bad)
        assert e.value.name == "SV_EINVAL"


def test_pauli_sum_checks(sv):
    h = I.xyz_chain(4)
    sv.check_pauli_sum(h, 4)
    with pytest.raises(sv.SvError):
        sv.check_pauli_sum(h, 5)
    bad = I.PauliSum(4, h.coeffs.copy(), h.paulis.copy())
    bad.paulis[0, 0] = ord("Q")
    with pytest.raises(sv.SvError):
        sv.check_pauli_sum(bad, 4)
    bad = I.PauliSum(4, h.coeffs.copy(), h.paulis.copy())
    bad.coeffs[3] = math.nan
    with pytest.raises(sv.SvError):
        sv.check_pauli_sum(bad, 4)


def test_no_device_is_reported(sv):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(sv.SvError) as e:
        sv.Context(0)
    assert e.value.name == "SV_ENODEV"


def test_autotune_rejects_bad_arguments(sv):
    L = sv.lib()
    cfg = sv._Config()
    assert L.sv_autotune(None, 0, 20, None, ctypes.byref(cfg)) == -1      # SV_EINVAL: no context
