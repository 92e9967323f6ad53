"""C-ABI library checks that need no GPU: it loads, exports every declared
symbol, and rejects bad arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "reedmd.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(reedmd_[a-z_0-9]+)\s*\(", txt)))


def _lib():
    from paper_0810_4737_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libreedmd.so not built")
    return _abi.load()


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("reedmd_create", "reedmd_run", "reedmd_destroy", "reedmd_sample_primaries",
                 "reedmd_debug_step", "reedmd_track_init", "reedmd_autotune", "reedmd_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    from paper_0810_4737_amd import _abi
    names = _declared()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_abi.EXPORTS)


def test_struct_sizes_match_header_layout():
    from paper_0810_4737_amd import _abi
    assert C.sizeof(_abi.Result) == 48
    assert _abi.RESULT_WORDS * 8 == C.sizeof(_abi.Result)
    assert C.sizeof(_abi.Species) == 8 + 4 * 8 + 8 * 8
    assert C.sizeof(_abi.Stopping) == 24
    assert _abi.STATS_WORDS * 8 == 10 * 8 + 8 * 8 + 5 * 8
    assert _abi.RECORD_WORDS == 32 + 9 * 216
    assert _abi.RECORD_WORDS_FLUORITE == 32 + 9 * 344
    # reedmd_run_params: 4 doubles, max_steps, seed, 2 ints, thresholds, 2 ints, bin_width,
    # 4 ints, cancel and track_log, track_log_cap, force_precision + range_mode,
    # vacancy + no_tail_handoff, r_cut
    assert C.sizeof(_abi.RunParams) == 4 * 8 + 8 + 8 + 8 + 8 + 8 + 8 + 16 + 16 + 8 + 8 + 8 + 8
    # reedmd_lattice: a, M2, sigma, Z2 + structure, M2b, sigma_b, Z2b + reserved
    assert C.sizeof(_abi.Lattice) == 3 * 8 + 8 + 2 * 8 + 8


def test_version_and_create_argument_errors_without_gpu():
    L = _lib()
    from paper_0810_4737_amd import _abi
    assert L.reedmd_version() == 100
    h = C.c_void_p()
    lat = _abi.Lattice(a=5.431, M2=28.0855, sigma=0.076, Z2=14, structure=0)
    pot = _abi.Potential(mode=0, s=1.0)
    stp = _abi.Stopping(mode=2, k=1.0)
    assert L.reedmd_create(None, C.byref(pot), C.byref(stp), C.byref(h)) == _abi.EINVAL
    bad = _abi.Lattice(a=-1.0, M2=28.0855, sigma=0.076, Z2=14, structure=0)
    assert L.reedmd_create(C.byref(bad), C.byref(pot), C.byref(stp), C.byref(h)) == _abi.EINVAL
    assert b"positive" in L.reedmd_last_error(None)
    badp = _abi.Potential(mode=0, s=0.0)
    assert L.reedmd_create(C.byref(lat), C.byref(badp), C.byref(stp), C.byref(h)) == _abi.EINVAL
    bads = _abi.Lattice(a=5.431, M2=28.0855, sigma=0.076, Z2=14, structure=3)
    assert L.reedmd_create(C.byref(bads), C.byref(pot), C.byref(stp), C.byref(h)) == _abi.EUNSUPPORTED
    # fluorite needs the anion species
    badf = _abi.Lattice(a=5.47, M2=238.03, sigma=0.05, Z2=92, structure=_abi.FLUORITE)
    assert L.reedmd_create(C.byref(badf), C.byref(pot), C.byref(stp), C.byref(h)) == _abi.EINVAL
    assert b"fluorite" in L.reedmd_last_error(None)
    assert L.reedmd_run(None, None, None, None, None, None, None) == _abi.EINVAL
    L.reedmd_destroy(None)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_0810_4737_amd import _abi
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _abi.load()


def test_binding_structs_match_the_c_header(tmp_path):
    """sizeof of every struct the binding mirrors, as the C compiler lays it out from the header."""
    import shutil
    import subprocess
    from paper_0810_4737_amd import _abi
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    names = {"reedmd_lattice": _abi.Lattice, "reedmd_potential": _abi.Potential,
             "reedmd_stopping": _abi.Stopping, "reedmd_species": _abi.Species, "reedmd_batch": _abi.Batch,
             "reedmd_sampler": _abi.Sampler, "reedmd_run_params": _abi.RunParams,
             "reedmd_result": _abi.Result, "reedmd_refine": _abi.Refine}
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include "reedmd.h"\nint main(void){\n' +
                   "".join(f'printf("{n} %zu\\n", sizeof({n}));\n' for n in names) + "return 0;}\n")
    exe = tmp_path / "sizes"
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if not os.path.exists(os.path.join(rocm, "include", "hip", "hip_runtime_api.h")):
        pytest.skip("HIP headers not found")
    subprocess.run([cc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"), "-I",
                    os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    got = dict(zip(out[0::2], map(int, out[1::2])))
    for n, cls in names.items():
        assert got[n] == C.sizeof(cls), (n, got[n], C.sizeof(cls))
