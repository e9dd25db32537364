"""Workgroup-size variants of the step kernel and the autotuner that picks
one per size bucket (worlds of different sizes batched in one call, Sec. 5.2):
every variant steps bitwise like the default, and the autotuner leaves the
model's state exactly as it found it."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_16536_amd import kamx, scenes  # noqa: E402

P = dict(dt=2e-3, eta=1e-4, rho_bilateral=1e-4, rho_contact=0.3, eps=1e-6, max_iters=200, torque_sigma=3.0,
         seed=17, log_restarts=0)


def hetero_model(n=12):
    scene = scenes.round_to_f32(scenes.heterogeneous_batch(n, seed=1003))
    return kamx.Model(scene, params=P)


def box_bin_model(n=6):
    scene = scenes.round_to_f32(scenes.box_bin_batch(n, seed=1005))
    m = kamx.Model(scene, params=dict(P, torque_sigma=0.0), max_contacts=64)
    m.contacts_box_bin(scenes.BIN_HALF, 0.01)
    return m


def snapshot(m):
    torch.cuda.synchronize()
    q, u = m.state()
    st = m.stats()
    return [q.cpu().numpy(), u.cpu().numpy(), m.impulses().cpu().numpy(), st["iters"].cpu().numpy(),
            st["status"].cpu().numpy(), np.array(m.reset_count())]


def assert_same(a, b, what):
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x, y), (what, k)


def test_bucket_table_and_validation():
    m = hetero_model()
    bks = m.buckets()
    print("\nbuckets:", bks, flush=True)
    assert [b["rows"] for b in bks] == [224, 96, 32]
    assert sum(b["worlds"] for b in bks) == 12
    for b in bks:
        assert b["threads"] == b["variants"][0]
        assert all(v % 64 == 0 and v >= 2 * b["rows"] for v in b["variants"])
    with pytest.raises(kamx.KamxError):
        m.set_bucket_threads(0, 256)     # the 224-row bucket needs two threads per row
    with pytest.raises(kamx.KamxError):
        m.set_bucket_threads(3, 128)     # no such bucket
    with pytest.raises(kamx.KamxError):
        m.autotune(0)
    with pytest.raises(kamx.KamxError):
        m.autotune(65)
    m.close()


@pytest.mark.parametrize("steps", [1, 20])
def test_every_variant_steps_like_the_default(steps):
    ref = hetero_model()
    ref.step(steps)
    want = snapshot(ref)
    bks = ref.buckets()
    ref.close()
    n_var = max(len(b["variants"]) for b in bks)
    for v in range(1, n_var):
        m = hetero_model()
        for bi, b in enumerate(bks):
            if v < len(b["variants"]):
                m.set_bucket_threads(bi, b["variants"][v])
        m.step(steps)
        assert_same(snapshot(m), want, f"variant {v}")
        m.close()


def test_box_bin_variants_step_alike():
    ref = box_bin_model()
    ref.step(30)
    want = snapshot(ref)
    (b,) = ref.buckets()
    ref.close()
    assert b["rows"] == 192 and len(b["variants"]) == 2
    m = box_bin_model()
    m.set_bucket_threads(0, b["variants"][1])
    m.step(30)
    assert_same(snapshot(m), want, "box bin")
    m.close()


@pytest.mark.parametrize("kind", ["hetero", "boxbin"])
def test_autotune_restores_the_state_and_keeps_a_variant(kind):
    make = hetero_model if kind == "hetero" else box_bin_model
    m = make()
    m.step(5)
    before = snapshot(m)
    ms = m.autotune(4)
    after = snapshot(m)
    assert_same(after, before, "state after autotune")
    bks = m.buckets()
    print(f"\n{kind}: autotune ms {ms}, chosen {[b['threads'] for b in bks]}", flush=True)
    for b, t in zip(bks, ms):
        assert b["threads"] in b["variants"]
        if len(b["variants"]) > 1:
            assert all(x > 0 for x in t)
            assert t[b["variants"].index(b["threads"])] == min(t)
    m.step(12)
    tuned = snapshot(m)
    m.close()
    # the same rollout without the autotuner, with the chosen sizes set by hand
    r = make()
    r.step(5)
    for bi, b in enumerate(bks):
        r.set_bucket_threads(bi, b["threads"])
    r.step(12)
    assert_same(snapshot(r), tuned, "continued rollout")
    r.close()
