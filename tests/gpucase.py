"""Shared helpers of the GPU parity tests: model cases and host/device copies."""
import numpy as np

H_CASES = {
    # name: (oracle kwargs, solver constructor kwargs, a)
    "symmetron_a1": (dict(model=0, a=1.0, lambda0=1.0, a_ssb=0.5),
                     ("symmetron", dict(lambda0=1.0, a_ssb=0.5)), 1.0),
    "symmetron_a05": (dict(model=0, a=0.5, lambda0=1.0, a_ssb=0.5),
                      ("symmetron", dict(lambda0=1.0, a_ssb=0.5)), 0.5),
    "fofr": (dict(model=1, a=1.0, n=1.0, fR0_abs=1e-5, omega_m=0.27, omega_l=0.73),
             ("fofr", dict(n=1.0, fR0_abs=1e-5, omega_m=0.27, omega_l=0.73)), 1.0),
    "fofr_a07": (dict(model=1, a=0.7, n=2.0, fR0_abs=1e-6, omega_m=0.3, omega_l=0.7),
                 ("fofr", dict(n=2.0, fR0_abs=1e-6, omega_m=0.3, omega_l=0.7)), 0.7),
    "linear": (dict(model=2, kappa=1.3, m2=0.4), ("linear", dict(kappa=1.3, m2=0.4)), 1.0),
    "linear_m0": (dict(model=2, kappa=0.8, m2=0.0), ("linear", dict(kappa=0.8, m2=0.0)), 1.0),
}


def models(name):
    from oracle import oracle as O
    from paper_1307_6748_amd import solver as S
    okw, (fn, skw), a = H_CASES[name]
    return O.Model(**okw), getattr(S, fn)(**skw), a


def field_for(name, n, seed):
    """A plausible iterate for the model (random, seeded)."""
    rng = np.random.default_rng(seed)
    if name.startswith("symmetron"):
        return rng.random((n, n, n))
    if name.startswith("fofr"):
        return -3.0 + 4.0 * rng.random((n, n, n))
    return rng.standard_normal((n, n, n))


def density(n, seed):
    rng = np.random.default_rng(seed)
    return 0.05 + 3.0 * rng.random((n, n, n)) ** 2


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def cubic(t, n):
    return host(t).reshape(n, n, n)
