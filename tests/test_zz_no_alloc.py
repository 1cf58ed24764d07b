"""The allocation-free residual entry point against isis_mg_residual.

isis_mg_residual_noalloc runs the same kernels with its scratch in a static
device array; its defect and RMS must equal those of the handle-based
isis_mg_residual bit for bit (same kernels, same grid, same fixed-order
reduction), also on a second call with a smaller grid (the array keeps the
first call's partial sums)."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpucase import dev, field_for, models

pytestmark = pytest.mark.gpu


def _noalloc(params, a, n, box, eta, phi, with_res=True):
    from paper_1307_6748_amd import _capi as A
    out = torch.full_like(eta, float("nan")) if with_res else None
    rms = C.c_double(float("nan"))
    pc = params.c()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = A.lib().isis_mg_residual_noalloc(
        C.byref(pc), float(a), n, float(box), C.c_void_p(eta.data_ptr()),
        C.c_void_p(phi.data_ptr()), None if out is None else C.c_void_p(out.data_ptr()),
        C.byref(rms), stream)
    assert rc == 0, A.lib().isis_mg_last_error(None).decode()
    return out, rms.value


@pytest.mark.parametrize("name", ["symmetron_a1", "fofr", "chameleon"])
def test_noalloc_residual_equals_handle_residual(name):
    from paper_1307_6748_amd import solver as S
    from paper_1307_6748_amd import synth
    om, sp, a = models(name)
    for n in (64, 32):  # second call smaller
        box = 2.0 * n
        eta = dev(synth.lognormal(n, box, 2.0, 300 + n))
        phi = dev(field_for(name, n, 301 + n))
        ref_out = torch.empty_like(eta)
        ref_rms = S.Solver(n, box).residual(eta, phi, sp, a, out=ref_out)
        out, rms = _noalloc(sp, a, n, box, eta, phi)
        torch.cuda.synchronize()
        assert rms == ref_rms, (n, rms, ref_rms)
        assert torch.equal(out, ref_out), n
        _, rms2 = _noalloc(sp, a, n, box, eta, phi, with_res=False)
        assert rms2 == ref_rms


def test_noalloc_residual_rejects_bad_sizes():
    from paper_1307_6748_amd import _capi as A
    from paper_1307_6748_amd import solver as S
    sp = S.symmetron()
    x = dev(np.ones((8, 8, 8)))
    pc = sp.c()
    rms = C.c_double()
    for n, box in ((8192, 1.0), (24, 1.0), (4, 1.0), (8, 0.0), (8, float("nan"))):
        rc = A.lib().isis_mg_residual_noalloc(C.byref(pc), 1.0, n, box, C.c_void_p(x.data_ptr()),
                                              C.c_void_p(x.data_ptr()), None, C.byref(rms), None)
        assert rc == A.ISIS_ERR_INVALID_ARG, (n, box)
        assert "residual_noalloc" in A.lib().isis_mg_last_error(None).decode()
