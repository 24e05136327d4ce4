"""The sampler front end on the GPU: every batch's images, ground-truth flow
fields and sampled densities equal the oracle's for the same pair ids and flow
fields; the captured-plan and eager schedules, and pre-fetching, give the same
batches; the full model, histogram adjustment and particle reuse follow the
oracle through the sampler."""

import numpy as np
import pytest
import torch

from oracle import epilogue as oep
from oracle import histogram as oh
from oracle import ra32
from oracle import seed as osd
from workloads.configs import Workload

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2512_09664_amd as sp
    from paper_2512_09664_amd import sampler as smp
    from gpu_util import to_np

BASE = dict(image_shape=(96, 128), batch_size=4, flows_per_batch=2, batches_per_flow=2,
            seeding_density=(0.03, 0.06), diameter={"dist": "uniform", "range": [1.5, 3.5]},
            blur={"radius": 1, "sigma": 0.7}, noise_sigma=0.0, bits=12, integrator="rk4", substeps=2,
            flow={"kind": "lamb_oseen", "grid_div": 4, "max_disp": 5.0}, seed=11)


def _wl(c):
    return Workload(name="sampler", sizes=(tuple(c.image_shape),), ppp=tuple(c.seeding_density), d_dist=c.d_dist,
                    d_params=c.d_params, I0=tuple(c.intensity), z=tuple(c.z), sheet_sigma=c.sheet.get("sigma", 0.5),
                    dt=c.dt, integrator=c.integrator, substeps=c.substeps, blur_radius=c.blur["radius"],
                    blur_sigma=c.blur["sigma"], bits=c.bits, seed=c.seed)


def _take(cfg, n):
    s = smp.make(cfg)
    out = []
    for _ in range(n):
        b = next(s)
        torch.cuda.synchronize()
        out.append({"i1": to_np(b.images1.contiguous()), "i2": to_np(b.images2.contiguous()),
                    "f": to_np(b.flow_fields), "ppp": to_np(b.params["seeding_densities"]),
                    "ids": b.params["pair_ids"], "fi": b.params["flow_index"], "ep": b.params["flow_epoch"]})
    s.close()
    return s, out


@pytest.mark.parametrize("use_graph", [True, False])
def test_batches_match_oracle(use_graph):
    cfg = smp.SamplerConfig.from_any({**BASE, "use_graph": use_graph})
    s, batches = _take(cfg, 3)
    wl = _wl(cfg)
    H, W = cfg.image_shape
    for b in batches:
        grids = s.flows.grids(b["ep"])
        for i in range(cfg.batch_size):
            flow = grids[b["fi"][i]]
            pid = int(b["ids"][i])
            ref = ra32.generate_pair_noiseless(wl, 0, flow, H, W, pair_id=pid)
            assert np.array_equal(b["i1"][i], ref["codes"][0]) and np.array_equal(b["i2"][i], ref["codes"][1])
            assert np.array_equal(b["f"][i], ra32.flow_field(flow, H, W))
            ppp, _, _ = osd.pair_scalars(H, W, *cfg.seeding_density, pid, cfg.seed)
            assert b["ppp"][i] == ppp


def test_schedules_and_prefetch_agree():
    outs = []
    for use_graph, prefetch in ((True, True), (False, True), (True, False)):
        cfg = smp.SamplerConfig.from_any({**BASE, "use_graph": use_graph, "prefetch": prefetch})
        outs.append(_take(cfg, 3)[1])
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            for k in ("i1", "i2", "f", "ppp"):
                assert np.array_equal(a[k], b[k])


def test_full_model_batch_matches_mirror():
    m = {**BASE, "rho": (-0.5, 0.5), "jitter": (0.1, 0.05, 0.02), "hide_p": 0.15,
         "sheet": {"law": "remark1", "dz0": 1.1, "shape": 1.5}}
    cfg = smp.SamplerConfig.from_any(m)
    s, batches = _take(cfg, 2)
    H, W = cfg.image_shape
    model = dict(ppp=cfg.seeding_density, d_dist=cfg.d_dist, d_params=cfg.d_params, I0=cfg.intensity, z=cfg.z,
                 rho=cfg.rho, anisotropic=True, jitter=cfg.jitter, hide_p=cfg.hide_p, d_max=cfg.d_max,
                 law="remark1", sheet_sigma=0.5, dz0=1.1, shape=1.5, dt=cfg.dt, substeps=cfg.substeps,
                 integrator=cfg.integrator)
    for b in batches:
        grids = s.flows.grids(b["ep"])
        for i in range(cfg.batch_size):
            ref = ra32.generate_pair_model(model, H, W, int(b["ids"][i]), cfg.seed, grids[b["fi"][i]], None,
                                           oep.blur_weights(1, 0.7), 12)
            assert np.array_equal(b["i1"][i], ref["codes"][0]) and np.array_equal(b["i2"][i], ref["codes"][1])


def test_histogram_adjustment_through_sampler():
    rng = np.random.default_rng(5)
    target = rng.integers(1, 50, 4096).astype(np.int64)
    cfg = smp.SamplerConfig.from_any({**BASE, "histogram": target.tolist()})
    s, batches = _take(cfg, 1)
    wl = _wl(cfg)
    H, W = cfg.image_shape
    b = batches[0]
    grids = s.flows.grids(0)
    for i in range(cfg.batch_size):
        ref = ra32.generate_pair_noiseless(wl, 0, grids[b["fi"][i]], H, W, pair_id=int(b["ids"][i]))
        assert np.array_equal(b["i1"][i], oh.match(ref["codes"][0], target, 12))
        assert np.array_equal(b["i2"][i], oh.match(ref["codes"][1], target, 12))


def test_particle_reuse_chain_matches_mirror():
    cfg = smp.SamplerConfig.from_any({**BASE, "batches_per_flow": 4, "particle_reuse": {"dt": 0.5, "batches": 3},
                                      "bits": 0, "blur": {"radius": 0, "sigma": 0.7}})
    s, batches = _take(cfg, 4)
    H, W = cfg.image_shape
    grids = s.flows.grids(0)
    for i in range(cfg.batch_size):
        flow = grids[batches[0]["fi"][i]]
        P = ra32.seed_pair(H, W, sp.particle_count(H, W, cfg.seeding_density[1]), cfg.seeding_density, i, cfg.seed,
                           cfg.d_dist, cfg.d_params, cfg.intensity, cfg.z)
        x1, y1 = P["x"], P["y"]
        for k in range(3):                          # batches 0, 1, 2 share the particles of batch 0
            x2, y2 = ra32.advect(flow, H, W, x1, y1, cfg.dt, cfg.substeps, cfg.integrator)
            for f, (xf, yf) in enumerate(((x1, y1), (x2, y2))):
                ref = ra32.render(xf, yf, P["z"], P["d"], P["I0"], H, W, 0.5)
                got = batches[k]["i1" if f == 0 else "i2"][i]
                assert np.array_equal(got, ref), f"batch {k} pair {i} frame {f}"
            x1, y1 = ra32.advect(flow, H, W, x2, y2, 0.5, cfg.substeps, cfg.integrator)
        # batch 3 is seeded afresh with its own pair ids
        pid = int(batches[3]["ids"][i])
        P3 = ra32.seed_pair(H, W, sp.particle_count(H, W, cfg.seeding_density[1]), cfg.seeding_density, pid,
                            cfg.seed, cfg.d_dist, cfg.d_params, cfg.intensity, cfg.z)
        assert np.array_equal(batches[3]["i1"][i], ra32.render(P3["x"], P3["y"], P3["z"], P3["d"], P3["I0"], H, W,
                                                                0.5))
