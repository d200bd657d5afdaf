"""Saving and restoring plans (numpy .npz).

A plan is fully determined by what it was built from (rank count, row starts,
variant, ranks per node, node map) and every rank's halo: building is
deterministic.  ``save_plan`` writes those and, for checking, every per-rank
array of every field; ``load_plan`` rebuilds the plan on the GPU from the
halos (``hx_plan_from_halos``) and, unless told not to, checks that each
field equals the saved one, raising ``ValueError`` otherwise.
"""
from __future__ import annotations

import numpy as np

from . import _lib as L

FORMAT = 1


def save_plan(plan: L.Plan, path) -> None:
    d = L.hx_plan_describe(plan)
    arrays = {"format": np.int64(FORMAT), "nranks": np.int64(d["nranks"]), "n": np.int64(d["n"]),
              "variant": np.int64(d["variant"]), "ppn": np.int64(d["ppn"]),
              "node_map": np.int64(L.NODE_MAPS[d["node_map"]]), "row_starts": d["row_starts"]}
    for f in L.FIELDS:
        off, vals = L.hx_plan_field_all(plan, f)
        arrays[f"{f}__off"] = off
        arrays[f] = vals
    np.savez(path, **arrays)


def load_plan(path, stream=None, verify: bool = True) -> L.Plan:
    import torch
    z = np.load(path, allow_pickle=False)
    if int(z["format"]) != FORMAT:
        raise ValueError(f"{path}: plan format {int(z['format'])}, expected {FORMAT}")
    R = int(z["nranks"])
    halo_ptr = z["halo__off"]
    halo = torch.from_numpy(np.ascontiguousarray(z["halo"])).to("cuda")
    plan = L.hx_plan_from_halos(R, z["row_starts"], int(z["ppn"]), int(z["variant"]), halo_ptr, halo,
                                stream=stream, node_map=int(z["node_map"]))
    if verify:
        for f in L.FIELDS:
            off, vals = L.hx_plan_field_all(plan, f)
            if not (np.array_equal(off, z[f"{f}__off"]) and np.array_equal(vals, z[f])):
                raise ValueError(f"{path}: field {f} of the rebuilt plan differs from the saved one")
    return plan
