"""Helpers of the GPU parity tests: upload seeded scenes, run the HIP library
through its C ABI, run the oracle on the same rays, compare."""
import numpy as np

import oracle
import scenegen

# decisions closer than this to their switching point are legitimately
# ambiguous between two correct double-precision implementations
AMBIG = {oracle.M_TGAP_PRI: 1e-10, oracle.M_RHO_PRI: 1e-9, oracle.M_TGAP_SEC: 1e-10, oracle.M_RHO_SEC: 1e-9,
         oracle.M_ENV: 1e-10, oracle.M_LOBE: 1e-10, oracle.M_COS: 1e-10, oracle.M_TMIN: 1e-10}


def torch():
    import torch as T
    return T


def dev(a, dtype=None):
    T = torch()
    return T.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype or T.float32)


def upload_scene(tr, scene):
    T = torch()
    ts = dict(mu=dev(scene.mu), q=dev(scene.q), scale=dev(scene.scale), opacity=dev(scene.opacity),
              albedo=dev(scene.albedo), roughness=dev(scene.roughness), metallic=dev(scene.metallic))
    tr.set_scene(**ts, object_offset=list(scene.object_offset))
    return ts


def state_args(tr, scene, state):
    M = scene.n_objects
    R = dev(state.R.reshape(M, 3, 3)) if M else None
    t = dev(state.t.reshape(M, 3)) if M else None
    return dict(env=dev(state.env), R=R, t=t)


def ambiguous(margins, include_secondary=True):
    keys = [oracle.M_TGAP_PRI, oracle.M_RHO_PRI, oracle.M_TMIN]
    if include_secondary:
        keys += [oracle.M_TGAP_SEC, oracle.M_RHO_SEC, oracle.M_ENV, oracle.M_LOBE, oracle.M_COS]
    amb = np.zeros(margins.shape[0], bool)
    for k in keys:
        amb |= margins[:, k] < AMBIG[k]
    return amb


def oracle_flags(flags):
    return int(flags) & (0xF | oracle.NEE | oracle.SOBOL)


def run_oracle(scene, state, o, d, ids, k, spp, seed, flags, threads=0, lists=True):
    sa = oracle.SceneArrays(scene, state.R, state.t, state.env)
    p = oracle.Params(k=k, spp=spp, seed=seed, flags=oracle_flags(flags))
    return oracle.render(sa, o, d, ids, p, lists=lists, threads=threads)


def rel_close(gpu, ref, rtol, floor_frac=1e-3):
    """max |gpu - ref| / max(|ref|, floor) with floor = floor_frac * mean |ref|."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    floor = floor_frac * max(float(np.abs(ref).mean()), 1e-30)
    err = np.abs(gpu - ref) / np.maximum(np.abs(ref), floor)
    return float(err.max()) if err.size else 0.0


GRAD_TOL = 1e-3  # relative, norm-wise per tensor and element-wise with a floor of 1e-3 * max|ref|


def grad_check(g_gpu, g_ref, name, tol=GRAD_TOL, nonzero=False):
    """Gradient parity: |a - b| <= tol |b| norm-wise, and element-wise
    |a_i - b_i| <= tol * max(|b_i|, 1e-3 max|b|).  Prints both errors and
    the worst element."""
    a = np.asarray(g_gpu, np.float64).ravel()
    b = np.asarray(g_ref, np.float64).ravel()
    nb = np.linalg.norm(b)
    if nonzero:
        assert nb > 0, name
    if nb == 0:
        assert np.abs(a).max(initial=0.0) == 0, name
        return
    floor = 1e-3 * np.abs(b).max()
    err = np.abs(a - b) / np.maximum(np.abs(b), floor)
    i = int(np.argmax(err))
    print(f"{name}: norm-wise {np.linalg.norm(a - b) / nb:.2e}, element-wise {err.max():.2e} "
          f"(element {i}: gpu {a[i]:.6e} ref {b[i]:.6e}, max|ref| {np.abs(b).max():.3e})", flush=True)
    assert np.linalg.norm(a - b) <= tol * nb, (name, np.linalg.norm(a - b) / nb)
    assert err.max() <= tol, (name, err.max(), i)
