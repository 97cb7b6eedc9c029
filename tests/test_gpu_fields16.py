"""u and sigma of the 16-bit storages are kept in 16 bits: BF16 rounded to nearest even, or FP16
holding the value times 2^12. The host round trip and the fields a step writes are checked
against those roundings computed here with numpy; their effect on the results is bounded by the
oracle comparisons of the 16-bit storages (test_gpu_precision_size, test_gpu_parity)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def bf16_rne(v):
    b = np.asarray(v, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def f16_scaled(v):
    return (np.asarray(v, dtype=np.float32) * np.float32(4096.0)).astype(np.float16).astype(np.float64) / 4096.0


ROUND = {"bf16": bf16_rne, "f16": f16_scaled}


def box(storage):
    from paper_1107_4889_amd import lbrbc

    nx, ny, nz = 70, 6, 5                # two column segments per row, the second ragged
    solid = np.zeros((nz, ny, nx), np.uint8)
    cfg = dict(nx=nx, ny=ny, nz=nz, periodic=(1, 1, 1), tau0=0.8, g_ext=(1e-5, 0.0, 0.0), storage=storage)
    return lbrbc.Simulation(cfg, solid), solid.size, cfg


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_field_round_trip(storage):
    sim, n, _ = box(storage)
    rng = np.random.default_rng(7)
    u = rng.uniform(-0.2, 0.2, (n, 3)) * 10.0 ** rng.uniform(-6, 0, (n, 1))
    s = rng.uniform(-1e-3, 1e-3, (n, 6)) * 10.0 ** rng.uniform(-5, 0, (n, 1))
    print(f"{storage}: field round trip on {n} nodes", flush=True)
    sim.lb_set_fields(u=u, sigma=s)
    d = sim.lb_get_fields(f=False, u=True, sigma=True)
    assert np.array_equal(d["u"], ROUND[storage](u))
    assert np.array_equal(d["sigma"], ROUND[storage](s))


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_step_writes_rounded_fields(storage):
    """After steps of a body-force-driven box the fields are values of the 16-bit format, and
    they round the FP32-storage fields of the same state to within the format's spacing."""
    sim, n, cfg = box(storage)
    # populations perturbed around rest (D3Q19 weights: rest, six axis, twelve diagonal speeds),
    # so that u and sigma vary from node to node
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None]
    f0 = w * (1.0 + 2e-3 * np.random.default_rng(3).standard_normal((19, n)))
    sim.lb_set_fields(f=f0)
    print(f"{storage}: 20 steps", flush=True)
    sim.lb_step(20)
    d = sim.lb_get_fields(f=True, u=True, sigma=True)
    for k in ("u", "sigma"):
        assert np.array_equal(d[k], ROUND[storage](d[k])), k
    assert np.abs(d["u"]).max() > 1e-5 and np.abs(d["sigma"]).max() > 1e-7
    # the same populations in FP32 storage: one step gives FP32 fields, which the 16-bit
    # fields of one step from the same populations round
    from paper_1107_4889_amd import lbrbc

    ref = lbrbc.Simulation(dict(cfg, storage="f32"), np.zeros((5, 6, 70), np.uint8))
    ref.lb_set_fields(f=d["f"])
    ref.lb_step(1)
    sim.lb_set_fields(f=d["f"])
    sim.lb_step(1)
    a, b = sim.lb_get_fields(f=False), ref.lb_get_fields(f=False)
    rel = 2.0 ** -8 if storage == "bf16" else 2.0 ** -11
    for k in ("u", "sigma"):
        scale = np.abs(b[k]).max()
        # FP16 below its normal range (2^-14 / 2^12) has an absolute spacing of 2^-36
        tol = rel * np.abs(b[k]) + (2.0 ** -36 if storage == "f16" else 0.0) + 1e-6 * scale
        assert (np.abs(a[k] - b[k]) <= tol).all(), k
