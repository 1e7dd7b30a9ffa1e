"""In situ rendering of a running simulation: zero-copy sources read from the
simulation's own tensors, a secondary field derived in update() and copied
(non-persistent), frames rendered every n-th step.

A frame rendered in situ must equal, bit for bit, the frame rendered from
host copies of the same field state through the ordinary upload path (layout
invariance), and match the oracle on those copies.
"""

import numpy as np
import pytest

import oracle
from parity import compare, log
from scenes import Scene, configs, make_source

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1611_09048_amd import Context
    assert torch.cuda.is_available()
    c = Context(device=0, stream=torch.cuda.current_stream())
    yield c
    c.close()


def scene_of(sim, tfs, width, height, direction):
    """The simulation's current fields as a host scene (the oracle's input)."""
    rho = sim.rho.cpu().numpy()
    e = sim.E.cpu().numpy()
    sim.derive_current()
    j = sim.J.cpu().numpy()
    n = sim.n
    srcs = [make_source("density", rho, guard=1, chain="", weight=0.6, tf=tfs[0]),
            make_source("E", e, guard=1, chain="length", weight=0.8, tf=tfs[1]),
            make_source("J", j, guard=1, chain="length | mul(2) | pow(0.5)", weight=0.9, tf=tfs[2])]
    return Scene(dims=(n, n, n), sources=srcs, camera=configs.orbit_camera((n, n, n), direction), width=width,
                 height=height, step=0.5, interpolation=1)


def test_insitu_frames_match_host_copies_and_oracle(ctx):
    import torch
    from paper_1611_09048_amd import device, insitu
    sim = insitu.FieldSimulation(n=40, seed=3)
    r = insitu.InSituRenderer(ctx, sim, volume_id=1)
    w, h = 96, 72
    img = torch.full((h, w, 4), float("nan"), device="cuda")
    dirs = [configs.D0, (-0.5, 0.7, 0.2)]

    def make_desc(frame):
        sc = scene_of_cam(frame)
        return device.render_job(sc, 1, img)

    def scene_of_cam(frame):
        n = sim.n
        return Scene(dims=(n, n, n), sources=[], camera=configs.orbit_camera((n, n, n), dirs[frame % 2]),
                     width=w, height=h, step=0.5, interpolation=1)

    st = r.run(steps=6, every=3, make_desc=make_desc)
    assert st.frames == 2 and sim.steps == 6
    # update() ran once per source per frame, in source order, enabled
    assert r.updates == [(0, 1), (1, 1), (2, 1)] * 2
    insitu_img = img.cpu().numpy()
    # the same state through the ordinary upload path, and the oracle
    sc = scene_of(sim, r.tfs, w, h, dirs[1])
    ref, _ = device.render_scene(ctx, sc, volume_id=2, count=False)
    log(f"in situ vs host copy: max |diff| = {np.abs(insitu_img - ref).max():.3e}")
    assert np.array_equal(insitu_img, ref)
    compare(insitu_img.reshape(-1, 4), None, oracle.render(sc, threads=8), label="in situ frame vs oracle")
    assert st.overhead > 0.0


def test_insitu_shared_scratch_for_two_secondary_fields(ctx):
    """Two non-persistent sources derived in turn into ONE scratch buffer by their
    update() callbacks (Sec. 3.2): the library copies each before the next
    update reuses the buffer, so the frame equals the one from separate copies."""
    import torch
    from paper_1611_09048_amd import binding, device, insitu
    sim = insitu.FieldSimulation(n=24, seed=5)
    for _ in range(2):
        sim.step()
    scratch = torch.zeros_like(sim.E)
    inner = (slice(1, -1),) * 3
    calls = []

    def update(user, enabled, pointer):
        k = int(user or 0)
        calls.append(k)
        if k in (1, 2):
            scratch[inner] = sim._curl(sim.B if k == 1 else sim.E)
            sim._fill_guards(scratch)
            torch.cuda.current_stream().synchronize()

    cb = binding.UPDATE_FN(update)
    rng = np.random.default_rng(9)
    tfs = [configs.random_tf(rng, 6, 0.05) for _ in range(3)]
    chains = ["", "length", "length | mul(3) | pow(0.5)"]
    descs = []
    for k, (t, f_dim) in enumerate(((sim.rho, 1), (scratch, 3), (scratch, 3))):
        comp, stride = insitu._accessor(t, f_dim)
        d = binding.source_desc(name=f"s{k}", f_dim=f_dim, dtype="f32", comp=comp, stride=stride, guard=1,
                                chain=chains[k], weight=0.8, persistent=(k == 0))
        d.update = cb
        d.user = k
        descs.append(d)
    ctx.set_sources(4, (24, 24, 24), descs)
    for k in range(3):
        ctx.set_transfer(4, k, tfs[k])
    cam = configs.orbit_camera((24, 24, 24), configs.D0)
    sc = Scene(dims=(24, 24, 24), sources=[], camera=cam, width=64, height=48, step=0.5, interpolation=1)
    img = torch.zeros((48, 64, 4), device="cuda")
    ctx.render([device.render_job(sc, 4, img)])
    torch.cuda.synchronize()
    assert calls == [0, 1, 2]
    # reference: the three fields as separate host copies through the upload path
    fields_ = []
    for k in (1, 2):
        scratch[inner] = sim._curl(sim.B if k == 1 else sim.E)
        sim._fill_guards(scratch)
        fields_.append(scratch.cpu().numpy())
    ref_sc = sc.with_(sources=[make_source("s0", sim.rho.cpu().numpy(), guard=1, chain=chains[0], weight=0.8,
                                           tf=tfs[0]),
                               make_source("s1", fields_[0], guard=1, chain=chains[1], weight=0.8, tf=tfs[1]),
                               make_source("s2", fields_[1], guard=1, chain=chains[2], weight=0.8, tf=tfs[2])])
    ref, _ = device.render_scene(ctx, ref_sc, volume_id=5, count=False)
    assert np.array_equal(img.cpu().numpy(), ref)
    compare(ref.reshape(-1, 4), None, oracle.render(ref_sc, threads=8), label="shared scratch vs oracle")
