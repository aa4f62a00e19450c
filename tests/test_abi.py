"""Host-side checks of the C-ABI library (no GPU needed).

The library must load and export every function include/sphcell.h declares;
host-only calls (version, status strings, defaults, footprint, argument
errors) are exercised without touching a device.
"""
import ctypes as C
import os
import re

import pytest

import paper_1309_3783_amd as sph
from paper_1309_3783_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sphcell.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = sph.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_host_only_calls():
    L = sph.lib()
    assert b"gfx950" in L.sph_version()
    assert L.sph_status_str(-4).startswith(b"h outgrew")
    p = sph.params()
    # Section III-B constants as defaults
    assert p.n_split == 400 and abs(p.split_frac - 0.875) < 1e-7
    assert p.n_target == 48.0 and abs(p.gamma - 5 / 3) < 1e-6 and p.alpha == 2.0
    assert sph.footprint(1_000_000) > 100 * 1_000_000
    with pytest.raises(sph.SphError):
        sph.footprint(-1)


def test_null_arguments_are_rejected():
    L = sph.lib()
    assert L.sph_tree_create(None, None) == binding.SPH_E_ARG
    assert L.sph_build_cells(None, None, None, None) == binding.SPH_E_ARG
    assert L.sph_density(None, None, None) == binding.SPH_E_ARG
    assert L.sph_force(None, None, None) == binding.SPH_E_ARG
    assert L.sph_run_graph(None, None, 1, None, None, None) == binding.SPH_E_ARG
    L.sph_ctx_destroy(None)


def test_integration_calls_reject_bad_arguments():
    import ctypes as C
    L = sph.lib()
    assert L.sph_kick(None, 0, 0.1, *([None] * 12)) == binding.SPH_E_ARG
    assert L.sph_drift(None, 1, None, None, 0.1, *([None] * 6)) == binding.SPH_E_ARG
    dt = C.c_double(0.0)
    assert L.sph_cfl_dt(None, 0, None, None, 0.3, C.byref(dt)) == binding.SPH_E_ARG


def test_context_creation_failure_is_explained():
    import ctypes as C
    L = sph.lib()
    h = C.c_void_p()
    st = L.sph_ctx_create(C.byref(h), 1 << 20, None)
    msg = L.sph_last_error(None).decode()
    # no GPU here: the device count fails; with one: the index is out of range
    assert (st == binding.SPH_E_HIP and msg.startswith("hipGetDeviceCount")) or \
        (st == binding.SPH_E_ARG and "out of range" in msg)
    assert not h.value


def test_workspace_size_host_only():
    L = sph.lib()
    b1 = sph.workspace_size(1_000_000, 1)
    b8 = sph.workspace_size(8_000_000, 1)
    assert b8 > 7 * (b1 - (32 << 20))          # grows with n
    assert sph.workspace_size(1000, 256) > sph.workspace_size(1000, 1)   # and with the set count
    assert sph.footprint(12345) == sph.workspace_size(12345, 1)
    out = C.c_size_t(0)
    assert L.sph_workspace_size(-1, 1, None, C.byref(out)) == binding.SPH_E_ARG
    assert L.sph_workspace_size(10, 0, None, C.byref(out)) == binding.SPH_E_ARG
    assert L.sph_tree_set_workspace(None, None, None, 0) == binding.SPH_E_ARG
    assert L.sph_tree_workspace_needed(None, C.byref(out)) == binding.SPH_E_ARG
    assert L.sph_build_cells_static(None, None, None, None) == binding.SPH_E_ARG


def _header_text():
    return open(os.path.join(ROOT, "include", "sphcell.h")).read()


def test_params_struct_matches_the_header():
    # the ctypes mirror of sph_params lists the header's fields in order,
    # with arrays of the same length
    src = re.sub(r"/\*.*?\*/", "", _header_text(), flags=re.S)
    body = re.search(r"typedef struct \{(.*?)\} sph_params;", src, flags=re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        m = re.match(r"(\w+)\s+(\w+)(?:\[(\d+)\])?$", decl)
        assert m, decl
        fields.append((m.group(2), int(m.group(3)) if m.group(3) else 1))
    mirror = [(n, getattr(t, "_length_", 1)) for n, t in binding.sph_params._fields_]
    assert fields == mirror


def test_flag_values_match_the_header():
    defs = dict(re.findall(r"#define (SPH_FLAG_\w+) (\d+)u", _header_text()))
    assert set(defs) == {"SPH_FLAG_PAIR_HASH", "SPH_FLAG_RESUME", "SPH_FLAG_NO_BLOCK_SKIP", "SPH_FLAG_SORTED_ONLY"}
    for name, v in defs.items():
        assert getattr(binding, name) == int(v), name


def test_counters_reject_a_null_context():
    L = sph.lib()
    assert L.sph_last_work(None, None, None) == binding.SPH_E_ARG
    assert L.sph_last_reads(None, None, None) == binding.SPH_E_ARG
