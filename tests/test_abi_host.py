"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/feti.h declares, validates meshes before touching the device and
fails loudly (FETI_EDEVICE) when no GPU is present.  No compute calls."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from workloads import config_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1508_02599_amd import feti
    if not os.path.exists(feti.LIB_PATH):
        pytest.skip("libfeti.so not built")
    return feti


def test_exports_every_declared_symbol():
    feti = _lib()
    hdr = open(os.path.join(ROOT, "include", "feti.h")).read()
    declared = set(re.findall(r"\b(feti_[a-z_]+)\s*\(", hdr))
    assert declared == set(feti.EXPORTED)
    lib = C.CDLL(feti.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


@pytest.mark.parametrize("mutate,msg", [
    (lambda m: setattr(m, "elem_sub", np.where(m.elem_sub == 3, 2, m.elem_sub)), "empty subdomain"),
    (lambda m: m.hex8.__setitem__((0, 0), 10**9), "out of range"),
    (lambda m: setattr(m, "dir_dof", m.dir_dof[:0]) or setattr(m, "dir_val", m.dir_val[:0]), "singular"),
    (lambda m: m.xyz.__setitem__((1, 1), np.nan), "non-finite"),
    (lambda m: m.mat.__setitem__((0, 2), 0.5), "bad linear material"),
    (lambda m: setattr(m, "dir_dof", np.concatenate([m.dir_dof, m.dir_dof[:1]])) or
     setattr(m, "dir_val", np.concatenate([m.dir_val, m.dir_val[:1]])), "duplicate"),
])
def test_setup_rejects_bad_mesh(mutate, msg):
    feti = _lib()
    m = config_mesh("cube8_s2")
    mutate(m)
    with pytest.raises(feti.FetiError) as ei:
        feti.Problem(m)
    assert ei.value.status == feti.FETI_EINVAL
    assert msg in str(ei.value)


def test_disconnected_subdomain_rejected():
    feti = _lib()
    m = config_mesh("cube8_s2")
    # move one corner element of subdomain 0 into subdomain 7 (not adjacent to it)
    m.elem_sub = m.elem_sub.copy()
    m.elem_sub[0] = 7
    with pytest.raises(feti.FetiError) as ei:
        feti.Problem(m)
    assert "disconnected" in str(ei.value)


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device path")
def test_valid_mesh_without_gpu_fails_loudly():
    feti = _lib()
    with pytest.raises(feti.FetiError) as ei:
        feti.Problem(config_mesh("cube8_s2"))
    assert ei.value.status == feti.FETI_EDEVICE


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device path")
def test_q2_meshes_pass_validation():
    """Q2 (27-node) cube and tube meshes pass the host-side plan builder (the
    failure is the missing device, after the plan is built); a Q2 mesh with
    4-node pressure faces is refused before the library is called."""
    from workloads import cube_mesh, tube_mesh
    feti = _lib()
    for m in (cube_mesh(4, 2, order=2), tube_mesh(1, 16, 4, sub=(1, 4, 2), order=2)):
        with pytest.raises(feti.FetiError) as ei:
            feti.Problem(m)
        assert ei.value.status == feti.FETI_EDEVICE
    m = tube_mesh(1, 16, 4, sub=(1, 4, 2), order=2)
    m.pface = m.pface[:, [0, 2, 8, 6]]
    with pytest.raises(ValueError):
        feti.Problem(m)
