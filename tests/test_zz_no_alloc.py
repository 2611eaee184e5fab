"""The conservation total without allocation (mifvm_conservation_static)
through the C-ABI against mifvm_conservation: bitwise equal on two calls in
a row, the second on a smaller state, and on a batch and an FP32 state."""
import ctypes as C

import numpy as np
import pytest

import synth
from conftest import cube

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2203_00925_amd.binding")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _static(st):
    out = C.c_double()
    lib = B.lib()
    lib.mifvm_conservation_static.restype = C.c_int
    lib.mifvm_conservation_static.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_void_p]
    rc = lib.mifvm_conservation_static(st._h, C.byref(out), B._stream(None))
    assert rc == 0, lib.mifvm_last_error().decode()
    return out.value


def _state(m, precision=B.FP64, seed=0):
    st = B.State(B.Mesh.from_cube(m), precision=precision)
    u = np.random.default_rng(seed).uniform(0.5, 2.0, len(m.tets))
    st.set_field(B.FIELD_U, torch.as_tensor(u, device="cuda"))
    return st


def test_static_conservation_equals_workspace_version():
    big = _state(cube(12, 1), seed=1)                    # 10,368 cells
    small = _state(cube(4, 2), seed=2)                   # 384 cells
    print("[gpu] static conservation: large then small state", flush=True)
    for st in (big, small, big):
        a, b = _static(st), st.conservation()
        assert a == b, (a, b)
    st32 = _state(cube(6, 3), precision=B.FP32, seed=3)
    assert _static(st32) == st32.conservation()
    meshes = [cube(4, 5), cube(5, 6), cube(6, 7)]           # 384, 750 and 1,296 cells
    batch = B.State(B.Mesh.from_batch(meshes))
    u = np.random.default_rng(4).uniform(0.5, 2.0, sum(len(m.tets) for m in meshes))
    batch.set_field(B.FIELD_U, torch.as_tensor(u, device="cuda"))
    assert _static(batch) == batch.conservation()
