"""Host-side checks of the HIP library that need no GPU: it loads, exports
every function include/rtm.h declares, and its host-only helpers (status
text, stability limit) agree with the oracle's behaviour."""
import pathlib
import re

import numpy as np
import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]


def _declared_functions():
    src = (ROOT / "include" / "rtm.h").read_text()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rtm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2001_06444_amd import rtm

    if not rtm.LIB_PATH.exists():
        pytest.fail("librtm.so is not built (run __graft_entry__.build())")
    return rtm.lib()


def test_library_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_every_declared_symbol():
    from paper_2001_06444_amd import rtm

    assert set(_declared_functions()) == set(rtm.SIGNATURES)


def test_status_strings(lib):
    for code in range(0, -9, -1):
        s = lib.rtm_status_str(code).decode()
        assert s and s != "unknown status"
    assert lib.rtm_status_str(5).decode() == "unknown status"


def test_cfl_limit_value_and_brute_force_agreement():
    """The library's stability limit (closed form from its stencil weights)
    is the one at which the FP64 oracle turns unstable: just below it a
    periodic box stays bounded for 10^4 steps, just above it blows up."""
    import oracle
    from paper_2001_06444_amd import rtm

    lim = rtm.cfl_limit()
    assert abs(lim - 0.784368) < 1e-5
    assert abs(rtm.cfl_number(1500.0, 1e-3, 10.0, 10.0) - 1500 * 1e-3 * np.sqrt(2) / 10) < 1e-6
    n, h, v = 32, 10.0, 2500.0
    u0 = np.random.default_rng(3).standard_normal((n, n))
    growth = {}
    for f in (0.995, 1.005):
        dt = f * lim / (v * np.sqrt(2.0) / h)
        out = oracle.forward(np.full((n, n), v), None, None, [], dz=h, dx=h, dt=dt, nb=0, nt=10000,
                             periodic=True, final=True, init=np.stack([u0, u0]))
        growth[f] = np.abs(out["final"][0]).max() / np.abs(u0).max()
    assert np.isfinite(growth[0.995]) and growth[0.995] < 1e3
    assert not np.isfinite(growth[1.005]) or growth[1.005] > 1e6
