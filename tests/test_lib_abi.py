"""CPU checks of the C ABI: the library loads, exports every declared symbol, and
rejects malformed input before touching a device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tpm.h")
LIB = os.path.join(ROOT, "paper_2001_07158_amd", "libtpm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(tpm_[a-z_]+)\s*\(", text)
    return sorted(set(n for n in names if not n.endswith("_t")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtpm.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), f"{n} declared in tpm.h but not exported"


def test_binding_covers_header():
    from paper_2001_07158_amd import tpm
    assert set(declared_functions()) <= set(tpm.EXPORTED)


def test_version_and_error_strings():
    from paper_2001_07158_amd import tpm
    assert "gfx950" in tpm.tpm_version()
    assert tpm.tpm_last_error() == ""


@pytest.mark.parametrize("bad", ["src", "dst", "tau", "color", "n"])
def test_malformed_graph_rejected_on_host(bad):
    from paper_2001_07158_amd import tpm
    n = 5
    src = np.array([0, 1, 2], dtype=np.int32)
    dst = np.array([1, 2, 3], dtype=np.int32)
    tau = np.array([1, 2, 3], dtype=np.int32)
    color = np.zeros(n, dtype=np.int32)
    if bad == "src":
        src[1] = n
    elif bad == "dst":
        dst[0] = -1
    elif bad == "tau":
        tau[2] = 0
    elif bad == "color":
        color[3] = 7
    elif bad == "n":
        n = 0
        color = np.zeros(0, dtype=np.int32)
    with pytest.raises(tpm.TpmError) as ei:
        tpm.tpm_graph_create(n, src, dst, tau, color, 2)
    assert ei.value.code == tpm.TPM_EINVAL
    assert tpm.tpm_last_error() != ""


def test_bad_tile_options_rejected():
    from paper_2001_07158_amd import tpm
    z = np.zeros(1, dtype=np.int32)
    with pytest.raises(tpm.TpmError) as ei:
        tpm.tpm_graph_create(2, z, z + 1, z + 1, np.zeros(2, dtype=np.int32), 1, tile_edges=5000)
    assert ei.value.code == tpm.TPM_EINVAL


def test_null_handles_are_errors():
    from paper_2001_07158_amd import tpm
    tpm.tpm_graph_destroy(None)  # NULL-safe
    with pytest.raises(tpm.TpmError):
        tpm.tpm_graph_stats_get(None)
    with pytest.raises(tpm.TpmError):
        tpm.tpm_decide(None, [0, 1], 1)
    for call in (lambda: tpm.tpm_graph_retile(None, 256), lambda: tpm.tpm_autotune(None, 4),
                 lambda: tpm.tpm_optimum_time(None, [0, 1], 1),
                 lambda: tpm.tpm_graph_sd(None, 0, 1),
                 lambda: tpm.tpm_static_sieve(None, [0, 1], 1),
                 lambda: tpm.tpm_graph_prune_static(None, [0, 1], 1),
                 lambda: tpm.tpm_extract_optimum(None, [0, 1], 1)):
        with pytest.raises(tpm.TpmError) as ei:
            call()
        assert ei.value.code == tpm.TPM_EINVAL


def test_unknown_creation_flags_rejected():
    from paper_2001_07158_amd import tpm
    z = np.zeros(1, dtype=np.int32)
    with pytest.raises(tpm.TpmError) as ei:
        tpm.tpm_graph_create(2, z, z + 1, z + 1, np.zeros(2, dtype=np.int32), 1, flags=0x4)
    assert ei.value.code == tpm.TPM_EINVAL


@pytest.mark.parametrize("case", ["neg_transit", "overflow", "neg_delay"])
def test_bad_delay_options_rejected_on_host(case):
    from paper_2001_07158_amd import tpm
    src, dst = np.array([0], np.int32), np.array([1], np.int32)
    kw = {}
    tau = np.array([2], np.int32)
    if case == "neg_transit":
        kw["transit"] = np.array([-1], np.int32)
    elif case == "overflow":
        tau = np.array([2**31 - 1], np.int32)
        kw["transit"] = np.array([1], np.int32)
    else:
        kw["delay"] = np.array([0, -1, 0], np.int32)
    with pytest.raises(tpm.TpmError) as ei:
        tpm.tpm_graph_create(3, src, dst, tau, np.zeros(3, np.int32), 1, **kw)
    assert ei.value.code == tpm.TPM_EINVAL


def test_library_resolves_its_own_symbols(lib):
    """Every symbol of the library's own namespace is defined in the library (a
    declaration mismatch between translation units would leave one undefined)."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--undefined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    assert "_ZN3tpm" not in out, [l for l in out.splitlines() if "_ZN3tpm" in l]
