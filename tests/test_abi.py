"""C-ABI checks that need no GPU: the library loads, exports every declared entry
point, validates configurations, and its FP64 host tables agree with the oracle."""
import ctypes
import re

import numpy as np
import pytest

import paper_1301_0322_amd as cola
from oracle import cosmology as cosmo


def _declared_functions():
    text = open(cola.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cola_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = cola.lib()
    names = _declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    # and the binding wraps each of them
    assert set(names) == set(cola._PROTOS)


def test_plan_validation():
    with pytest.raises(cola.ColaError) as e:
        cola.Plan(cola.Config(np=20, nm=40))
    assert e.value.status == -2
    with pytest.raises(cola.ColaError):
        cola.Plan(cola.Config(np=32, nm=48))        # nm not a multiple of np
    with pytest.raises(cola.ColaError):
        cola.Plan(cola.Config(n_lpt=0.0))
    with pytest.raises(cola.ColaError):
        cola.Plan(cola.Config(a_init=1.0, a_final=0.5))
    with pytest.raises(cola.ColaError):
        cola.Plan(cola.Config(n_steps=0))
    with pytest.raises(cola.ColaError):
        cola.Plan(cola.Config(flags=0x80))
    assert cola.lib().cola_strerror(-2).decode().startswith("unsupported size")


def test_workspace_size():
    # four nm^3 float meshes, the per-step binning buffers (8 + 4 bytes per
    # particle, tile-count arrays, halo faces of every tile) and two tile-sorted
    # copies of the particle state (2 x 13 words per particle)
    for np_side, nm in ((32, 64), (64, 64), (256, 512)):
        with cola.Plan(cola.Config(np=np_side, nm=nm)) as p:
            meshes = 4 * nm**3 * 4
            extra = p.workspace_bytes() - meshes - 104 * np_side**3
            assert 12 * np_side**3 < extra < 12 * np_side**3 + 0.4 * nm**3 * 4


def _oracle_scheme(flags: int) -> dict:
    """Oracle Config fields for the library's variant flags."""
    out = {"log_a_steps": bool(flags & cola.COLA_FLAG_LOG_A_STEPS), "u1_drift": bool(flags & cola.COLA_FLAG_U1_DRIFT)}
    if flags & cola.COLA_FLAG_NO_LPT_FRAME:
        out["scheme"] = "pm"
    elif flags & cola.COLA_FLAG_KDK_STD:
        out["scheme"] = "standard"
    return out


@pytest.mark.parametrize("kw", [{}, {"n_steps": 3}, {"omega_m": 0.25, "omega_l": 0.75}, {"n_lpt": 1.5},
                                {"omega_m": 0.3, "omega_l": 0.6},
                                {"flags": cola.COLA_FLAG_KDK_STD},
                                {"flags": cola.COLA_FLAG_NO_LPT_FRAME, "n_steps": 7},
                                {"flags": cola.COLA_FLAG_LOG_A_STEPS},
                                {"flags": cola.COLA_FLAG_KDK_STD | cola.COLA_FLAG_LOG_A_STEPS, "a_init": 0.02},
                                {"flags": cola.COLA_FLAG_U1_DRIFT},
                                {"flags": cola.COLA_FLAG_U1_DRIFT | cola.COLA_FLAG_LOG_A_STEPS, "n_lpt": 1.5}])
def test_host_step_table_matches_oracle(kw):
    cfg = cola.Config(**kw)
    with cola.Plan(cfg) as p:
        t = p.step_table()
    ocfg = cosmo.Config(**{k: v for k, v in kw.items() if k != "flags"}, **_oracle_scheme(kw.get("flags", 0)))
    ot = cosmo.step_table(ocfg)
    g = ot.grow
    np.testing.assert_allclose(t["a"], ot.a, rtol=1e-14)
    for col in ("D1", "D2", "TD1", "TD2", "T2D1", "T2D2"):
        np.testing.assert_allclose(t[col], g[col], rtol=1e-9, err_msg=col)
    np.testing.assert_allclose(t["alpha"], ot.alpha, rtol=1e-10)
    np.testing.assert_allclose(t["beta"][:-1], ot.beta, rtol=1e-10)
    np.testing.assert_allclose(t["dD1"][:-1], ot.dD1, rtol=1e-8)
    np.testing.assert_allclose(t["dD2"][:-1], ot.dD2, rtol=1e-8)
    np.testing.assert_allclose(t["a_mid"][:-1], ot.a_mid, rtol=1e-14)
    np.testing.assert_allclose(t["force"], 1.5 * ocfg.omega_m * ot.a, rtol=1e-14)


def test_binding_rejects_host_buffers_before_the_call():
    # the binding checks device, dtype, contiguity and size before a pointer reaches
    # the library (which receives bare pointers and cannot check sizes)
    import torch
    with cola.Plan(cola.Config(np=16, nm=32)) as p:
        s = torch.zeros(3, 16**3)
        with pytest.raises(ValueError, match="CUDA"):
            p.density(s, torch.zeros(32**3), s)
        with pytest.raises(ValueError, match="CUDA"):
            p.run(torch.zeros(16**3), cola.Particles(s, s, s, s), s, s, s)


def test_ensemble_checks_every_noise_before_the_call():
    # the ensemble graph bakes in bare pointers: every member's noise is checked (a
    # CUDA tensor of at least np^3 floats) before anything is allocated or captured
    import torch
    plans = [cola.Plan(cola.Config(np=16, nm=32)), cola.Plan(cola.Config(np=24, nm=48))]
    try:
        with pytest.raises(ValueError, match="noises\\[0\\].*CUDA"):
            cola.Ensemble(plans, [torch.zeros(16**3), torch.zeros(24**3)])
        with pytest.raises(ValueError, match="one per member"):
            cola.Ensemble(plans, [torch.zeros(16**3)])
        with pytest.raises(ValueError, match="one per member"):
            cola.Ensemble([], [])
    finally:
        for p in plans:
            p.close()


def test_density_noalloc_rejects_sizes_beyond_its_scratch():
    # 512^3 particles need 1.6 GB of binning buffers, more than the 256 MiB static
    # scratch: rejected with COLA_ERR_WORKSPACE before any device call (the pointers
    # are never touched)
    with cola.Plan(cola.Config(np=512, nm=1024, box=400.0)) as p:
        assert cola.lib().cola_density_noalloc(p._c, 1, 1, None) == -6
        assert "static scratch" in cola.lib().cola_strerror(-6).decode()
    with cola.Plan(cola.Config(np=16, nm=32)) as p:
        assert cola.lib().cola_density_noalloc(p._c, None, 1, None) == -1
        assert cola.lib().cola_density_noalloc(None, 1, 1, None) == -1


def test_fft_rotation_setting():
    """Rotated planes: off by default below nm = 1024, on at 1024; the rotation is the x
    pass's inner DFT length (rows per plane); only -1, 0 and 1 are accepted."""
    with cola.Plan(cola.Config(np=16, nm=32)) as p:
        assert p.get_fft_rotation() == 0
        for bad in (-2, 2, 8):
            with pytest.raises(cola.ColaError):
                p.set_fft_rotation(bad)
        p.set_fft_rotation(1)
        assert p.get_fft_rotation() == 8
        p.set_fft_rotation(-1)
        assert p.get_fft_rotation() == 0
    with cola.Plan(cola.Config(np=128, nm=768)) as p:
        assert p.get_fft_rotation() == 0
        p.set_fft_rotation(1)
        assert p.get_fft_rotation() == 24
    with cola.Plan(cola.Config(np=512, nm=1024, box=400.0)) as p:
        assert p.get_fft_rotation() == 32
        p.set_fft_rotation(0)
        assert p.get_fft_rotation() == 0


def test_resident_steps_setting():
    with cola.Plan(cola.Config(np=16, nm=32)) as p:
        p.set_resident_steps(1)
        p.set_resident_steps(0)
        for bad in (-1, 2):
            with pytest.raises(cola.ColaError):
                p.set_resident_steps(bad)
