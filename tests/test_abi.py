"""The C-ABI library loads without a GPU and exports every symbol that
include/helm.h declares (no compute calls here)."""

import ctypes
import os
import re

import pytest

from paper_1809_03808_amd import helm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "helm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(helm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("helm_setup", "helm_solve", "helm_report_get", "helm_residual", "helm_destroy",
              "helm_strerror", "helm_eig1d", "helm_default_options"):
        assert n in names
    assert set(names) == set(helm.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(helm.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_strerror_and_defaults():
    assert helm.strerror(0) == "success"
    assert "singular" in helm.strerror(helm.HELM_ESINGULAR)
    opt = helm.Options()
    helm.lib().helm_default_options(ctypes.byref(opt))
    assert opt.precision == helm.PREC_FP64 and opt.tol == 1e-10 and opt.max_iter == 8 and opt.check == 1
    assert opt.transform == helm.TRANSFORM_FFT and opt.boundary == helm.BOUNDARY_AUTO
    assert opt.eigen == helm.EIGEN_AUTO


def test_setup_rejects_unknown_boundary_mode():
    with pytest.raises(helm.HelmError) as e:
        helm.Plan((8, 8, 8), (0.1,) * 3, 3.0, boundary=7)
    assert e.value.code == helm.HELM_EINVAL


def test_setup_rejects_unknown_eigen_mode():
    with pytest.raises(helm.HelmError) as e:
        helm.Plan((8, 8), (0.1,) * 2, 3.0, eigen=5)
    assert e.value.code == helm.HELM_EINVAL


@pytest.mark.parametrize("device", [False, True])
def test_eig1d_rejects_bad_arguments(device):
    # argument errors are returned before any device call
    for args in ((2, 0.5, 1.0), (8, 0.0, 1.0), (8, 0.1, float("nan"))):
        with pytest.raises(helm.HelmError) as e:
            helm.eig1d(*args, device=device)
        assert e.value.code == helm.HELM_EINVAL


@pytest.mark.parametrize("grid,h,omega,mask,code", [
    ((16, 16), (1 / 15, 1 / 15), 0.0, 0b1111, helm.HELM_ESINGULAR),
    ((16, 2), (1 / 15, 1.0), 3.0, 0b1111, helm.HELM_EINVAL),
    ((16, 16), (1 / 15, -1.0), 3.0, 0b1111, helm.HELM_EINVAL),
    ((16, 16), (1 / 15, 1 / 15), 3.0, 0b0011, helm.HELM_EUNSUPPORTED),  # last axis all Neumann
    ((16, 16, 16), (0.1,) * 3, float("nan"), 0b111111, helm.HELM_EINVAL),
])
def test_setup_argument_errors(grid, h, omega, mask, code):
    """Validation happens on the host before any device call."""
    with pytest.raises(helm.HelmError) as e:
        helm.Plan(grid, h, omega, mask)
    assert e.value.code == code


def test_batch_create_rejects_bad_arguments():
    import ctypes
    L = helm.lib()
    out = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 1)(None)
    assert L.helm_batch_create(None, 1, 1, ctypes.byref(out)) == helm.HELM_EINVAL
    assert L.helm_batch_create(arr, 0, 1, ctypes.byref(out)) == helm.HELM_EINVAL
    assert L.helm_batch_create(arr, 1, 0, ctypes.byref(out)) == helm.HELM_EINVAL
    assert L.helm_batch_solve(None, None, None, None, None) == helm.HELM_EINVAL
    L.helm_batch_destroy(None)


def test_dense_transform_size_limit():
    """DENSE needs every periodised length <= HELM_DENSE_MAX (checked before
    any device call); an unknown transform code is rejected."""
    n = helm.DENSE_MAX + 1
    with pytest.raises(helm.HelmError) as e:
        helm.Plan((n, 16), (1.0 / (n - 1), 1 / 15), 5.0, transform=helm.TRANSFORM_DENSE)
    assert e.value.code == helm.HELM_EUNSUPPORTED
    with pytest.raises(helm.HelmError) as e:
        helm.Plan((16, 16), (1 / 15, 1 / 15), 5.0, transform=7)
    assert e.value.code == helm.HELM_EINVAL


@pytest.mark.parametrize("grid", [(16, 4098), (16, 8193), (131073, 16), (262145, 16), (16, 140000, 9)])
def test_setup_size_limits(grid):
    """Lengths beyond this build's limits are refused before any device call:
    a line axis above 4097 nodes, a periodised length whose transform would
    need more than two passes of 512."""
    h = tuple(1.0 / (n - 1) for n in grid)
    with pytest.raises(helm.HelmError) as e:
        helm.Plan(grid, h, 5.0)
    assert e.value.code == helm.HELM_EUNSUPPORTED


@pytest.mark.parametrize("c,faces,code", [
    (0.0, ((0.0, 0.0), (0.0, 0.0)), helm.HELM_ESINGULAR),          # Neumann Laplace: constants
    (float("nan"), ((1.0, 1.0), (1.0, 1.0)), helm.HELM_EINVAL),
    (-1.0, ((1.0, float("inf")), (1.0, 1.0)), helm.HELM_EINVAL),
    (9.0, ((1.0, 1.0), (1.0, 1.0)), helm.HELM_EUNSUPPORTED),        # c > 0, real faces: resonance possible
    (-4.0, ((-2j, 3j), (-1j, -1j)), helm.HELM_EUNSUPPORTED),        # imaginary parts of both signs
    (-4.0, ((1.0, 1.0), (-0.5, 1.0)), helm.HELM_EUNSUPPORTED),      # negative real g
    (0.0, ((1.0, 1.0), (0.0, 0.0)), helm.HELM_EUNSUPPORTED),        # Laplace, Neumann last axis
    (4.0, ((-2j, -2j), (0.0, 0.0)), helm.HELM_EUNSUPPORTED),        # real faces on the last axis, c > 0
])
def test_setup_general_rejects_coefficients(c, faces, code):
    """helm_setup_general's coefficient checks run before any device call."""
    with pytest.raises(helm.HelmError) as e:
        helm.Plan((8, 8), (1 / 7, 1 / 7), 2.0, faces, c=c)
    assert e.value.code == code


def test_face_coefficients_follow_helm_setup():
    assert helm.face_coefficients(3.0, ((True, False), (0.5 - 1j, True))) == [0.0, -3.0, 0.0, 0.0, 0.5, -1.0, 0.0, -3.0]
