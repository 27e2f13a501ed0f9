"""The C ABI library loads and exports every symbol include/ni.h declares (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "ni.h")


def declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ni_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["ni_params_default", "ni_create", "ni_destroy", "ni_set_stream", "ni_integrate", "ni_label",
              "ni_fill", "ni_irls", "ni_unet_load", "ni_status_str", "ni_last_error", "ni_abi_version"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2510_11508_amd as ni
    L = ni.lib()
    for n in declared():
        assert hasattr(L, n), n
    from paper_2510_11508_amd.binding import EXPORTED
    assert sorted(EXPORTED) == declared()


def test_host_only_calls():
    import paper_2510_11508_amd as ni
    L = ni.lib()
    p = ni.ni_params_default()
    assert (p.theta_c_deg, p.irls_iters, p.align_iters, p.out_L, p.out_U) == (2.0, 15, 2, 1e-5, 1e-3)
    assert p.cg_rtol == 1e-6 and p.connectivity == 4 and p.outlier_mode == 1
    assert p.q_rtol == 1e-5 and p.q_rtol_refine == 1e-5
    assert L.ni_params_default(None) == ni.NI_E_ARG
    assert L.ni_status_str(ni.NI_E_SHAPE) == b"output capacity too small"
    assert L.ni_abi_version() == 3
    assert L.ni_destroy(None) == ni.NI_E_ARG
    assert L.ni_integrate(None, None, None, 1, 1, None, None, None, None, None, 0, None, None) == ni.NI_E_ARG


def test_struct_layouts_match_header():
    from paper_2510_11508_amd import binding as B
    # field lists mirror the C structs in include/ni.h, in order
    src = re.sub(r"/\*.*?\*/", "", open(HDR).read(), flags=re.S)

    def fields(struct):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + struct + ";", src).group(1)
        out = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            typ, rest = decl.split(None, 1) if not decl.startswith("int") else (decl.split()[0], decl.split(None, 1)[1])
            for nm in rest.split(","):
                out.append(re.sub(r"\[.*\]", "", nm.strip()))
        return out

    for cls, name in [(B.ni_camera, "ni_camera"), (B.ni_params, "ni_params"), (B.ni_report, "ni_report")]:
        assert [f[0] for f in cls._fields_] == fields(name), name
