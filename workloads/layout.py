"""Order a workload's arrays and parameters the way the library's C ABI takes
them (include/opt.h).  Pure re-packaging: no arithmetic on the data."""
import numpy as np

ARRAY_ORDER = {
    "arap_warp": ["U", "C", "mask"],
    "poisson": ["T", "mask"],
    "sfs": ["D", "Im", "edge_r", "edge_c"],
    "flow": ["I", "Ihat", "Ihat_dx", "Ihat_dy"],
    "arap_mesh": ["U", "C"],
    "arap_volume": ["U", "C"],
    "laplacian": ["A"],
    "laplacian_graph": ["A"],
    "lp_smooth": ["A"],
    "intrinsic": ["I"],
}
# the library's name of each workload energy
LIB_ENERGY = {"laplacian_graph": "laplacian"}


def param_list(d):
    p = d["params"]
    e = d["energy"]
    if e in ("arap_warp", "arap_mesh", "arap_volume", "flow", "laplacian", "laplacian_graph"):
        return [p["w_fit"], p["w_reg"]]
    if e == "lp_smooth":
        return [p["w_fit"], p["w_reg"], p["p"], p["eps"]]
    if e == "intrinsic":
        return [p["w_fit"], p["w_a"], p["w_s"], p["p"], p["eps"]]
    if e == "poisson":
        return []
    if e == "sfs":
        return [p["w_p"], p["w_s"], p["w_g"], p["f_x"], p["f_y"], p["u_x"], p["u_y"], *p["L"]]
    raise ValueError(e)


def problem_args(d, bulk_dtype):
    """(energy, [numpy arrays], [params], dims) with bulk arrays cast to
    ``bulk_dtype`` and masks left as uint8.  ``dims`` holds width/height (and
    depth for a 3D grid) for a grid or n_vertices/edges for a graph."""
    e = d["energy"]
    arrs = []
    for k in ARRAY_ORDER[e]:
        a = np.asarray(d[k])
        arrs.append(np.ascontiguousarray(a if a.dtype == np.uint8 else a.astype(bulk_dtype)))
    if "V" in d:
        dims = dict(n_vertices=int(d["V"]), edges=np.ascontiguousarray(d["edges"], dtype=np.int32))
    elif e == "arap_volume":
        dims = dict(width=int(d["W"]), height=int(d["H"]), depth=int(d["D"]))
    else:
        dims = dict(width=int(d["W"]), height=int(d["H"]))
    return LIB_ENERGY.get(e, e), arrs, param_list(d), dims
