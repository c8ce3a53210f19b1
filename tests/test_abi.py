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
    return sorted(set(re.findall(r"\b(pns_[a-z0-9_]+)\s*\(", text)))


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


def test_sizes_beyond_the_largest_tile_are_rejected_before_q_is_read():
    """N above 16384 is PNS_EUNSUPPORTED for pns_create (also with the
    autotuner on, which prepares the matrix first), pns_create_batch and
    pns_autotune, before the matrix is read: the buffer passed here holds a
    single entry."""
    from paper_2210_10513_amd import binding as b
    Q = np.zeros(1, np.int16)
    for autotune in (0, 1):
        o = b.pns_opts_default()
        o.dtype = b.PNS_I16
        o.autotune = autotune
        with pytest.raises(b.PNSError) as ei:
            b.pns_create(Q, 16385, 0.1, 64, b.PNS_MODE_UNBIASED_SYS, o)
        assert ei.value.code == b.PNS_EUNSUPPORTED and "16384" in str(ei.value)
    probs = [b.pns_problem(Q=Q.ctypes.data, N=N, layout=0, subset_size=0, num_chains=2, L0=0, betas=None, beta=0.1)
             for N in (100, 20000)]
    o = b.pns_opts_default()
    o.dtype = b.PNS_I16
    with pytest.raises(b.PNSError) as ei:
        b.pns_create_batch(probs, b.PNS_MODE_UNBIASED_SYS, o)
    assert ei.value.code == b.PNS_EUNSUPPORTED and "problem 1" in str(ei.value)
    with pytest.raises(b.PNSError) as ei:
        b.pns_autotune(Q, 16385, 0.1, 0, b.PNS_MODE_UNBIASED_SYS, o)
    assert ei.value.code == b.PNS_EUNSUPPORTED


@pytest.mark.parametrize("kw,expect", [
    (dict(problems=0), "num_problems"),
    (dict(N=0), "N must be positive"),
    (dict(chains=0), "num_chains"),
    (dict(n=9, mode=2), "subset size"),
    (dict(beta=-2.0), "beta"),
    (dict(mode=5), "unknown mode"),
    (dict(layout=3), "unknown layout"),
    (dict(reserved=True), "reserved"),
])
def test_create_batch_rejects_bad_arguments(kw, expect):
    from paper_2210_10513_amd import binding as b
    Qs = [np.zeros((8, 8), np.int32), np.zeros((12, 12), np.int32)]
    probs = [b.pns_problem(Q=q.ctypes.data, N=q.shape[0], layout=0, subset_size=4, num_chains=2, L0=0,
                           betas=None, beta=0.1) for q in Qs]
    probs[1].N = kw.get("N", 12)
    probs[1].num_chains = kw.get("chains", 2)
    probs[1].beta = kw.get("beta", 0.1)
    probs[1].layout = kw.get("layout", 0)
    if "n" in kw:
        probs[0].subset_size = kw["n"]
    o = b.pns_opts_default()
    if kw.get("reserved"):
        o.reserved[6] = 1
    if kw.get("problems") == 0:
        probs = []
        ctx = ctypes.c_void_p()
        rc = b.lib.pns_create_batch(ctypes.byref(ctx), 0, None, 0, ctypes.byref(o))
        assert rc == b.PNS_EINVAL and expect in b.pns_last_error()
        return
    with pytest.raises(b.PNSError) as ei:
        b.pns_create_batch(probs, kw.get("mode", b.PNS_MODE_BASIC), o)
    assert ei.value.code == b.PNS_EINVAL
    assert expect in str(ei.value)


def test_autotune_rejects_bad_arguments():
    from paper_2210_10513_amd import binding as b
    Q = np.zeros((8, 8), np.int32)
    for n, mode, expect in ((9, b.PNS_MODE_BASIC, "subset size"), (-1, b.PNS_MODE_BASIC, "subset size"),
                            (4, 6, "unknown mode")):
        with pytest.raises(b.PNSError) as ei:
            b.pns_autotune(Q, 8, 0.1, n, mode)
        assert ei.value.code == b.PNS_EINVAL and expect in str(ei.value)


@pytest.mark.parametrize("field,value,expect", [
    ("dim", 0, "dim"), ("dim", 8, "dim"), ("pairs", 0, "pairs"), ("pairs", 33, "pairs"),
    ("sigma", 0.0, "sigma"), ("sigma", float("nan"), "sigma"), ("mu0", float("inf"), "mu0"),
    ("L0", 0, "L0"), ("num_chains", 0, "num_chains"), ("log_capacity", -1, "log_capacity"),
    ("sigma", 1e-200, "2 sigma^2"),
])
def test_continuous_create_rejects_bad_options(field, value, expect):
    from paper_2210_10513_amd import binding as b
    o = b.pns_cont_opts()
    b.lib.pns_cont_opts_default(ctypes.byref(o))
    assert (o.dim, o.pairs, o.mu0, o.sigma, o.L0, o.num_chains) == (2, 25, 9.0, 0.1, 1000, 1)
    setattr(o, field, value)
    ctx = ctypes.c_void_p()
    rc = b.lib.pns_cont_create(ctypes.byref(ctx), ctypes.byref(o))
    assert rc == b.PNS_EINVAL and expect in b.pns_last_error() and not ctx.value


def test_continuous_create_rejects_reserved_fields():
    from paper_2210_10513_amd import binding as b
    o = b.pns_cont_opts()
    b.lib.pns_cont_opts_default(ctypes.byref(o))
    o.reserved[3] = 1
    ctx = ctypes.c_void_p()
    assert b.lib.pns_cont_create(ctypes.byref(ctx), ctypes.byref(o)) == b.PNS_EINVAL
    assert "reserved" in b.pns_last_error()


def test_structs_match_header_layout(tmp_path):
    """Every struct of the binding has the size and field offsets that a C
    compiler gives the header's declaration."""
    import subprocess
    from paper_2210_10513_amd import binding as b
    structs = {"pns_opts": b.pns_opts, "pns_problem": b.pns_problem, "pns_problem_info": b.pns_problem_info,
               "pns_tune": b.pns_tune, "pns_chain_stats": b.pns_chain_stats, "pns_cont_opts": b.pns_cont_opts,
               "pns_class_profile": b.pns_class_profile}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pns.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, f"{name}.{fname}"


def test_checkpoint_calls_reject_null_arguments():
    from paper_2210_10513_amd import binding as b
    size = ctypes.c_int64(-1)
    assert b.lib.pns_save(None, None, 0, ctypes.byref(size)) == b.PNS_EINVAL
    assert b.lib.pns_load(None, None, 0) == b.PNS_EINVAL
    assert "NULL" in b.pns_last_error()
    n = ctypes.c_int32(0)
    assert b.lib.pns_profile(None, 1) == b.PNS_EINVAL
    assert b.lib.pns_profile_read(None, None, 0, ctypes.byref(n)) == b.PNS_EINVAL
    assert b.lib.pns_class_of_chain(None, None) == b.PNS_EINVAL
