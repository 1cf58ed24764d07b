"""Host-side checks of the C ABI: the library loads, exports every function
the header declares, and rejects invalid arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1307_6748_amd import _capi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "isis_mg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b(isis_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("isis_mg_create", "isis_mg_solve", "isis_mg_residual", "isis_mg_destroy"):
        assert n in names
    assert len(names) >= 14


def test_library_exports_every_declared_symbol():
    lib = A.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(n for n, _, _ in A.SIGNATURES) == declared_functions()


def _desc(**kw):
    d = A.DescC(64, 64.0, 2, 2, 32, 50, A.ISIS_FP64, 0.0, 0, None, None, 0)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_workspace_size_validation():
    lib = A.lib()
    ok = lib.isis_mg_workspace_size(C.byref(_desc()))
    assert ok > 0
    # bigger with the FP32 hierarchy of the mixed mode
    assert lib.isis_mg_workspace_size(C.byref(_desc(precision=A.ISIS_MIXED))) > ok
    assert lib.isis_mg_workspace_size(C.byref(_desc(precision=A.ISIS_MIXED,
                                                    fp32_floor=1e-7))) > ok
    for bad in (dict(N=12), dict(N=4), dict(box=0.0), dict(box=float("nan")),
                dict(nu_coarse=0), dict(max_cycles=0), dict(max_cycles=A.MAX_HIST),
                dict(precision=7), dict(temporal_block=3), dict(temporal_block=-2), dict(nu_pre=0, nu_post=0),
                dict(fp32_floor=-1e-6), dict(fp32_floor=2.0), dict(fp32_floor=1e-13),
                dict(fp32_floor=float("nan")), dict(guess_accept=-0.1),
                dict(guess_accept=1.5), dict(guess_accept=float("nan")),
                dict(restriction=2), dict(restriction=-2), dict(judge_skip=2),
                dict(judge_skip=-1), dict(nu_post=-2), dict(nu_pre=-1),
                dict(prolongation=2), dict(prolongation=-2)):
        assert lib.isis_mg_workspace_size(C.byref(_desc(**bad))) == 0, bad
    # nu_post = -1 picks the sweeps per model; with nu_pre = 0 that is still >= 1
    assert lib.isis_mg_workspace_size(C.byref(_desc(nu_pre=0, nu_post=-1))) > 0


def test_create_rejects_bad_workspace_without_gpu():
    lib = A.lib()
    h = C.c_void_p()
    assert lib.isis_mg_create(C.byref(_desc()), C.byref(h)) == A.ISIS_ERR_INVALID_ARG
    assert h.value is None
    assert b"workspace" in lib.isis_mg_last_error(None)
    assert lib.isis_mg_create(C.byref(_desc(N=10)), C.byref(h)) == A.ISIS_ERR_INVALID_ARG


@pytest.mark.parametrize("params,a", [
    (A.ModelParamsC(A.ISIS_SYMMETRON, 0.0, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0), 1.0),
    (A.ModelParamsC(A.ISIS_SYMMETRON, 1.0, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0), 0.0),
    (A.ModelParamsC(A.ISIS_SYMMETRON, 1.0, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0), float("nan")),
    (A.ModelParamsC(A.ISIS_FR_HS, 1.0, 0.5, 1, 1, 0.0, 0.27, 0.73, 1, 0), 1.0),
    (A.ModelParamsC(A.ISIS_FR_HS, 1.0, 0.5, 1, -1.0, 1e-5, 0.27, 0.73, 1, 0), 1.0),
    (A.ModelParamsC(A.ISIS_LINEAR, 1.0, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, -1.0), 1.0),
    (A.ModelParamsC(9, 1.0, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0), 1.0),
    # chameleon: alpha > 0, mu > 0, n > -1
    (A.ModelParamsC(A.ISIS_CHAMELEON, 1, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0, 0.0, 1.0, 1.0), 1.0),
    (A.ModelParamsC(A.ISIS_CHAMELEON, 1, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0, 1.0, -1.0, 1.0), 1.0),
    (A.ModelParamsC(A.ISIS_CHAMELEON, 1, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0, 1.0, 1.0, -1.0), 1.0),
    # the paper's f(R) variable is an f(R) option, 0 or 1
    (A.ModelParamsC(A.ISIS_SYMMETRON, 1, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0, 1, 1, 1, 1), 1.0),
    (A.ModelParamsC(A.ISIS_FR_HS, 1, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0, 1, 1, 1, 2), 1.0),
])
def test_ops_validate_params_on_host(params, a):
    lib = A.lib()
    rc = lib.isis_op_defect(C.byref(params), a, 8, 1.0, None, None, None, None, None)
    assert rc == A.ISIS_ERR_INVALID_ARG
    assert lib.isis_mg_last_error(None)


def test_ops_validate_sizes_on_host():
    lib = A.lib()
    p = A.ModelParamsC(A.ISIS_LINEAR, 1.0, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0)
    fake = C.c_void_p(256)  # never dereferenced: validation fails first
    assert lib.isis_op_halfsweep(C.byref(p), 1.0, 7, 1.0, fake, fake, None, 0, None) == -1
    assert lib.isis_op_halfsweep(C.byref(p), 1.0, 8, 1.0, fake, fake, None, 2, None) == -1
    assert lib.isis_op_restrict(5, fake, fake, None) == -1
    assert lib.isis_op_prolong_correct(2, fake, fake, fake, None) == -1
    assert lib.isis_op_prolong_correct_w(2, fake, fake, fake, None) == -1
    assert lib.isis_op_prolong_correct_w(6, fake, None, fake, None) == -1
    assert lib.isis_op_sweeps(C.byref(p), 1.0, 8, 1.0, fake, fake, fake, None, 1, 5, None) == -1
    assert lib.isis_op_cold_start(C.byref(p), 1.0, 0, None, None, None) == 0


def test_ops_reject_misaligned_pointers_on_host():
    """The kernels move z-neighbouring cells as 16-byte pairs: an array that
    is only 8-byte aligned is refused before anything is launched."""
    lib = A.lib()
    p = A.ModelParamsC(A.ISIS_LINEAR, 1.0, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0)
    ok, bad = C.c_void_p(4096), C.c_void_p(4096 + 8)  # never dereferenced
    assert lib.isis_op_defect(C.byref(p), 1.0, 8, 1.0, ok, bad, None, ok, None) == -1
    assert b"aligned" in lib.isis_mg_last_error(None)
    assert lib.isis_op_restrict(8, bad, ok, None) == -1
    assert lib.isis_op_prolong_correct(8, ok, ok, bad, None) == -1
    assert lib.isis_op_prolong_correct_w(8, ok, ok, bad, None) == -1
    assert lib.isis_op_halfsweep(C.byref(p), 1.0, 8, 1.0, ok, ok, bad, 0, None) == -1
    assert lib.isis_op_sweeps(C.byref(p), 1.0, 8, 1.0, ok, bad, ok, None, 1, 0, None) == -1
    assert lib.isis_op_fas_descend(C.byref(p), 1.0, 8, 1.0, ok, ok, None, ok, ok, ok, ok, bad,
                                   None, None) == -1
    assert lib.isis_op_fas_descend(C.byref(p), 1.0, 8, 1.0, ok, ok, None, ok, ok, ok, ok, ok,
                                   bad, None) == -1
    assert lib.isis_op_restrict_fw(8, ok, bad, None) == -1
    assert lib.isis_op_restrict_fw(7, ok, ok, None) == -1
    assert lib.isis_op_coarse_solve(C.byref(p), 1.0, 1.0, bad, ok, None, 4, None) == -1
    assert lib.isis_op_cold_start(C.byref(p), 1.0, 8, ok, bad, None) == -1


def test_force_validates_on_host():
    lib = A.lib()
    ok, bad = C.c_void_p(4096), C.c_void_p(4096 + 8)  # never dereferenced
    lin = A.ModelParamsC(A.ISIS_LINEAR, 1.0, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0)
    sym0 = A.ModelParamsC(A.ISIS_SYMMETRON, 1.0, 0.5, 1, 1, 1e-5, 0.0, 0.73, 1, 0)
    fr = A.ModelParamsC(A.ISIS_FR_HS, 1.0, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0)
    assert lib.isis_force(C.byref(lin), 1.0, 7, 1.0, None, ok, ok, ok, ok, None) == -1
    assert lib.isis_force(C.byref(lin), 1.0, 8, 0.0, None, ok, ok, ok, ok, None) == -1
    assert lib.isis_force(C.byref(sym0), 1.0, 8, 1.0, ok, None, ok, ok, ok, None) == -1
    assert b"Omega_m" in lib.isis_mg_last_error(None)
    assert lib.isis_force(C.byref(fr), 1.0, 8, 1.0, None, ok, ok, ok, ok, None) == -1
    cham = A.ModelParamsC(A.ISIS_CHAMELEON, 1, 0.5, 1, 1, 1e-5, 0.27, 0.73, 1, 0, 1.0, 1.0, 1.0)
    assert lib.isis_force(C.byref(cham), 1.0, 8, 1.0, ok, None, ok, ok, ok, None) == \
        A.ISIS_ERR_UNSUPPORTED
    assert b"chameleon" in lib.isis_mg_last_error(None)
    assert lib.isis_force(C.byref(fr), 1.0, 8, 1.0, ok, None, ok, bad, ok, None) == -1


def test_unet_training_parts_reject_bad_arguments_without_gpu():
    """The split training step (forward, backward, Adam) and the tensor
    accessor validate their arguments before any GPU work."""
    lib = A.lib()
    buf = C.c_void_p(256)  # never dereferenced: every call below fails validation
    P = C.c_void_p
    assert lib.isis_unet_forward(None, buf, buf, 1.0, 32, None, buf, 1 << 40, None) == \
        A.ISIS_ERR_INVALID_ARG
    assert lib.isis_unet_forward(buf, buf, buf, 1.0, 24, None, buf, 1 << 40, None) == \
        A.ISIS_ERR_INVALID_ARG
    assert lib.isis_unet_forward(buf, buf, buf, 0.0, 32, None, buf, 1 << 40, None) == \
        A.ISIS_ERR_INVALID_ARG
    small = lib.isis_unet_workspace_size(32, 1) - 1
    assert lib.isis_unet_forward(buf, buf, buf, 1.0, 32, None, buf, small, None) == \
        A.ISIS_ERR_INVALID_ARG
    assert lib.isis_unet_backward(buf, None, buf, 32, buf, 1 << 40, None, None, None) == \
        A.ISIS_ERR_INVALID_ARG
    assert lib.isis_unet_backward(buf, buf, buf, 32, buf, small, None, None, None) == \
        A.ISIS_ERR_INVALID_ARG
    for bad in ((None, buf, buf, buf, 10, 1, 1e-3), (buf, buf, buf, buf, -1, 1, 1e-3),
                (buf, buf, buf, buf, 10, 0, 1e-3), (buf, buf, buf, buf, 10, 1, -1.0)):
        assert lib.isis_unet_adam_step(*bad, None) == A.ISIS_ERR_INVALID_ARG, bad
    assert lib.isis_unet_adam_step(buf, buf, buf, buf, 0, 1, 1e-3, None) == A.ISIS_OK
    ptr, vox, ch = P(), C.c_long(), C.c_int()
    for bad in ((None, 32, 0), (buf, 24, 0), (buf, 32, -1), (buf, 32, 22)):
        assert lib.isis_unet_tensor(*bad, C.byref(ptr), C.byref(vox), C.byref(ch)) == \
            A.ISIS_ERR_INVALID_ARG, bad
    # the layout is host arithmetic: shapes of the tensors of a 32^3 workspace
    base = 1 << 20
    shapes = {}
    for tid in range(22):
        assert lib.isis_unet_tensor(C.c_void_p(base), 32, tid, C.byref(ptr), C.byref(vox),
                                    C.byref(ch)) == A.ISIS_OK
        shapes[tid] = (vox.value, ch.value, ptr.value)
    assert shapes[0][:2] == (32 ** 3, 16) and shapes[7][:2] == (4 ** 3, 64)
    assert shapes[8][:2] == (8 ** 3, 64) and shapes[12][:2] == (32 ** 3, 16)
    assert shapes[14][:2] == (32 ** 3, 16) and shapes[17][:2] == (4 ** 3, 64)
    assert shapes[18][:2] == (8 ** 3, 128) and shapes[20][:2] == (32 ** 3, 48)
    assert shapes[21][:2] == (32 ** 3, 1)
    ends = sorted((p, p + v * c * (4 if t == 21 else 2)) for t, (v, c, p) in shapes.items())
    assert all(b[0] >= a[1] for a, b in zip(ends, ends[1:]))  # disjoint
    assert ends[-1][1] <= base + lib.isis_unet_workspace_size(32, 1)
