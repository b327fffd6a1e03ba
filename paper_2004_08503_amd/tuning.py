"""Tile-shape tuning table.

The library compiles its kernels for IDP_DG_NUM_TILE_SHAPES tile shapes per
degree.  Every shape gives bitwise the same results; only the speed
differs, and it depends on the device.  `sweep()` measures the shapes on
the current device (idp_dg_tune on a representative state of each kernel
family and degree) and writes the choices to a JSON table next to the
library; `apply_solver` sets a handle's tile shape from that table (the
server does; a new handle otherwise keeps shape 0).

    python -m paper_2004_08503_amd.tuning        # sweep and write the table
"""
import json
import os
import sys
import time

from . import idp_dg, workloads as W

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_table.json")

# representative meshes: about a million nodes per degree, square
_NODES = 1 << 20


def _mesh_for(p):
    return max(4, int(round((_NODES / (p + 1) ** 2) ** 0.5)))


def _key(prob):
    return str(idp_dg.family_of(prob))


def load_table(path=TABLE_PATH):
    """The table, or None when there is none."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if not isinstance(t, dict) or "tile_shape" not in t:
        raise ValueError("%s is not a tuning table" % path)
    return t


def apply_solver(sv, table=None):
    """Set the Solver's tile shape from the table (no table, or no entry for
    its family and degree: keep the current shape).  Returns the shape."""
    table = load_table() if table is None else table
    if table:
        shape = table["tile_shape"].get(_key(sv.prob), {}).get(str(sv.prob.p))
        if shape is not None and shape != sv.tile_shape:
            sv.set_tile_shape(int(shape))
    return sv.tile_shape


def sweep(families=("euler", "burgers"), degrees=range(1, 9), reps=5, log=print):
    """Measure tile shapes per (family, degree) with idp_dg_tune on a
    representative state of about a million nodes; returns the table."""
    import torch
    table = {"tile_shape": {}, "device": torch.cuda.get_device_name(0),
             "measured": time.strftime("%Y-%m-%d")}
    for fam in families:
        for p in degrees:
            n = _mesh_for(p)
            wl = W.euler_2d(n=n, p=p) if fam == "euler" else W.burgers_2d(n=n, p=p)
            sv = idp_dg.Solver(wl.prob)
            u = torch.from_numpy(wl.u0).cuda()
            shape = sv.tune(u, wl.cfl, reps=reps)
            table["tile_shape"].setdefault(_key(wl.prob), {})[str(p)] = int(shape)
            log("tuning: %s p=%d %d^2: shape %d" % (fam, p, n, shape))
            sv.close()
            del u
    return table


def main():
    table = sweep(log=lambda m: print(m, file=sys.stderr, flush=True))
    with open(TABLE_PATH, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(json.dumps(table))


if __name__ == "__main__":
    main()
