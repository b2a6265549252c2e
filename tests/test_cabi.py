"""The C ABI without a GPU: the library loads, exports every function that
include/sparc_hip.h declares, the Python binding declares exactly those, and the
host-only entry points (status strings, density of states) work and match the
oracle.  CPU only: no device call is made."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1603_04339_amd import sparc as sp
from oracle.bands import dos as oracle_dos

HEADER = os.path.join(os.path.dirname(__file__), "..", "include", "sparc_hip.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|size_t|int64_t|char)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_symbols_exported_and_bound():
    names = _declared()
    assert len(names) > 40
    lib = sp.load()
    for n in names:
        assert hasattr(lib, n), f"{n} declared but not exported"
    assert sorted(sp.exported_symbols()) == names


def test_status_strings():
    lib = sp.load()
    for st in (sp.OK, sp.EINVAL, sp.ESHAPE, sp.ENOMEM, sp.ENOTSPD, sp.ENOCONV, sp.EDEVICE, sp.ENAN):
        s = lib.sparc_status_string(st)
        assert isinstance(s, bytes) and len(s) > 0


def test_dos_matches_oracle_and_rejects_bad_width():
    rng = np.random.default_rng(31)
    eig = np.sort(rng.uniform(-1, 1, (5, 7)), axis=1)
    wk = rng.uniform(0, 1, 5)
    wk /= wk.sum()
    E = np.linspace(-1.5, 1.5, 301)
    np.testing.assert_allclose(sp.dos(eig, wk, E, 0.03), oracle_dos(eig, wk, E, 0.03), rtol=1e-13, atol=1e-13)
    with pytest.raises(sp.SparcError) as e:
        sp.dos(eig, wk, E, 0.0)
    assert e.value.status == sp.EINVAL
