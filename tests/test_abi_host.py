"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
symbol the header declares, rejects bad arguments before touching a device, and its
frequency-to-time matrix matches the oracle's independent construction."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2109_00661_amd import binding as B
from paper_2109_00661_amd import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "rjsmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rjsmc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = declared_functions()
    assert "rjsmc_loglik" in names and "rjsmc_create" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) <= set(B._SIGS)


def test_create_rejects_bad_system_without_device():
    s = W.system()
    bad = dict(s)
    bad["freq_hz"] = s["freq_hz"][::-1].copy()          # decreasing
    with pytest.raises(B.RJSMCError) as e:
        B.Context(bad)
    assert e.value.status == B.RJSMC_E_INVALID
    bad = dict(s, kmax_cond=12, kmax_charg=8)            # > 16 merged layers
    with pytest.raises(B.RJSMCError) as e:
        B.Context(bad)
    assert e.value.status == B.RJSMC_E_INVALID
    assert "capacities" in B.lib().rjsmc_last_error().decode()


def test_time_kernel_matches_oracle(system, K_oracle):
    K = B.build_time_kernel(system["freq_hz"], system["gate_open_s"], system["gate_close_s"])
    # entrywise against the row scale, and the image of physical spectra
    row = np.abs(K_oracle).max(axis=1, keepdims=True)
    assert np.max(np.abs(K - K_oracle) / row) < 1e-11
    from oracle import em
    for p in (W.truth_three_layer(), W.merged_population(8, 5, seed=21)):
        for i in range(len(p["kappa"])):
            sig, ms, thick = em.merged_stack(p, i)
            G = em.secondary_hz(system, sig, ms, thick, 10 ** p["log10_tau"][i], p["c"][i]).imag
            y_lib, y_or = K @ G, K_oracle @ G
            scale = np.abs(K_oracle * G[None, :]).sum(axis=1)
            assert np.all(np.abs(y_lib - y_or) <= 2e-13 * scale), np.max(np.abs(y_lib - y_or) / scale)


def test_time_kernel_rejects_bad_gates():
    f = W.frequencies_hz()
    lo, hi = W.gate_edges_s()
    with pytest.raises(B.RJSMCError):
        B.build_time_kernel(f, hi, lo)
