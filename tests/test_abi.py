"""The C-ABI library loads and exports every function include/pns.h declares;
argument validation that needs no device rejects bad calls.  CPU only: no
compute call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pns.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pns_[a-z_]+)\s*\(", text)))


def test_header_declares_the_core_trio():
    names = declared_functions()
    for core in ("pns_create", "pns_run", "pns_read"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2210_10513_amd import binding
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    assert sorted(binding.EXPORTS) == declared_functions()


def test_version_and_defaults():
    from paper_2210_10513_amd import binding as b
    assert b.pns_version().count(".") == 2
    o = b.pns_opts_default()
    assert o.num_chains == 1 and o.L0 == 100 and o.launch == b.PNS_LAUNCH_PERSISTENT
    assert o.dtype == b.PNS_I32 and o.layout == b.PNS_SYMMETRIC


@pytest.mark.parametrize("kw,expect", [
    (dict(N=0), "N must be positive"),
    (dict(n=0, mode=1), "subset size"),
    (dict(n=9, mode=2), "subset size"),
    (dict(beta=-1.0), "beta"),
    (dict(beta=float("inf")), "beta"),
    (dict(mode=7), "unknown mode"),
    (dict(dtype=9), "unknown dtype"),
    (dict(layout=5), "unknown layout"),
    (dict(chains=0), "num_chains"),
    (dict(hist_big=True), "histograms"),
    (dict(reserved=True), "reserved"),
])
def test_create_rejects_bad_arguments(kw, expect):
    from paper_2210_10513_amd import binding as b
    N = kw.get("N", 8)
    Q = np.zeros((max(N, 1), max(N, 1)), np.int32)
    o = b.pns_opts_default()
    o.dtype = kw.get("dtype", b.PNS_I32)
    o.layout = kw.get("layout", b.PNS_SYMMETRIC)
    o.num_chains = kw.get("chains", 1)
    if kw.get("hist_big"):
        N = 30
        Q = np.zeros((N, N), np.int32)
        o.hist = 1
    if kw.get("reserved"):
        o.reserved[3] = 1
    with pytest.raises(b.PNSError) as ei:
        b.pns_create(Q, N, kw.get("beta", 0.1), kw.get("n", 4), kw.get("mode", b.PNS_MODE_RF), o)
    assert ei.value.code == b.PNS_EINVAL
    assert expect in str(ei.value)
