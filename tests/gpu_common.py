"""Helpers shared by the GPU tests: build a context for a list of replicas
and run the oracle on the same seeded inputs."""
import numpy as np

from paper_2201_04622_amd import inputs as I


def make_ctx(replicas, precision=0, lanes=4, block=256, knots=None):
    import torch

    import paper_2201_04622_amd.eamfe as E
    knots = knots or I.synthetic_eam_knots()
    ctx = E.Context(0, precision)
    ctx.set_launch(lanes, block)
    ctx.eam_setup(knots)
    arrs = I.batch_arrays(replicas)
    x0 = E.to_soa(arrs["x0"])
    ctx.system_setup(replicas, x0)
    return ctx, x0, arrs


def split(a, offsets):
    return [a[offsets[r]:offsets[r + 1]] for r in range(len(offsets) - 1)]


def rel_norm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*args):
    print(*args, flush=True)
