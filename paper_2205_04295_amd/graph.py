"""HIP-graph capture of whole reconstructions.

A call of the sweep is a fixed sequence of launches on one stream with no
allocation, no synchronisation and no memset (fills are kernels), so it can
be recorded once and replayed: the replay issues the whole lock-step sweep
(two launches per position and tick, for every job) as one graph launch.
Each replay continues the reconstruction from the current buffer contents.
"""
from __future__ import annotations

import torch

from . import api


def capture_batched(jobs, warmup=True, **params):
    """Record mrpie_rpie_batched(jobs, **params) into a CUDA/HIP graph.

    jobs: list of dicts (obj, probe, pos, intens[, err, status]); workspaces
    are allocated before capture and attached to the dicts.  Returns the
    torch.cuda.CUDAGraph; call .replay() to run it."""
    # allocate every workspace (and set kernel attributes) outside capture
    if warmup:
        snap = [(j["obj"].clone(), j["probe"].clone()) for j in jobs]
        wss = api.rpie_batched(jobs, **params)
        for j, ws, (o, p) in zip(jobs, wss, snap):
            j["workspace"] = ws
            j["obj"].copy_(o)
            j["probe"].copy_(p)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        api.rpie_batched(jobs, **params)
    return g


def capture_plain(obj, probe, pos, intens, workspace=None, err=None, **params):
    """Record one mrpie_rpie call (integer-crop sweep) into a graph."""
    nbytes = api.workspace_size(api.problem_of(obj, probe, pos), api.make_params(**params))
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=obj.device)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        api.rpie(obj, probe, pos, intens, err=err, workspace=workspace, **params)
    return g, workspace
