"""Helpers shared by the GPU tests: run the HIP path and the oracle on the
same seeded inputs and bring both results to numpy."""
import numpy as np
import scipy.sparse as sp

from inputs.rules import polygon_dirs


def make_config(w, **over):
    import paper_2207_03921_amd as nl
    d = dict(kernel=w["kernel"], c=float(w["c"]), delta=float(w["delta"]),
             outer_xi=w["outer"].xi, outer_w=w["outer"].w, inner_xi=w["inner"].xi,
             inner_w=w["inner"].w, approach=w.get("approach", "bary"),
             singular_n=int(w.get("singular_n", 0)), precision=w.get("precision", "fp64"),
             ansatz=w.get("ansatz", "cg"), material_c=w.get("material_c"))
    if d["approach"] == "poly":
        d["polygon_dirs"] = polygon_dirs(int(w.get("polygon_n", 32)))
    d.update(over)
    return nl.Config(**d)


def f_affine_of(w):
    if w.get("f_affine") is not None:
        return w["f_affine"]
    return [(float(v), 0.0, 0.0) for v in w["f"]]


def gpu_run(mesh, w, precision=None, export=True):
    """Pairs, pattern, values and load vector from the HIP library."""
    import torch
    import paper_2207_03921_amd as nl
    cfg = make_config(w, **({} if precision is None else {"precision": precision}))
    dm = nl.DeviceMesh.from_numpy(mesh)
    pairs = nl.nlfem_build_pairs(dm, cfg)
    info = nl.nlfem_pairs_info(pairs)
    out = {"info": info}
    if export:
        k, l, c = nl.nlfem_pairs_export(pairs)
        out["pairs"] = (k.cpu().numpy(), l.cpu().numpy(), c.cpu().numpy())
    rp, col = nl.nlfem_csr_pattern(pairs)
    val = nl.nlfem_assemble(dm, cfg, pairs)
    b = nl.nlfem_rhs(dm, cfg, f_affine=f_affine_of(w))
    torch.cuda.synchronize()
    out.update(row_ptr=rp.cpu().numpy(), col=col.cpu().numpy(), val=val[:info["nnz"]].cpu().numpy(),
               b=b.cpu().numpy())
    out["_keep"] = (dm, cfg, pairs)
    return out


def to_sparse(rp, col, val, n):
    return sp.csr_matrix((val, col, rp), shape=(n, n))


def rel_frob(A, B):
    d = (A - B)
    nb = np.sqrt((B.multiply(B)).sum()) if sp.issparse(B) else np.linalg.norm(B)
    nd = np.sqrt((d.multiply(d)).sum()) if sp.issparse(d) else np.linalg.norm(d)
    return float(nd / nb)


def entrywise(G, A):
    """Largest entry error of a row relative to the row's largest entry, over
    all rows: catches an error in small (far-field) entries that the
    Frobenius norm of the whole matrix would hide under the diagonal."""
    D = abs(G - A).tocsr()
    Aa = abs(A).tocsr()
    dmax = np.asarray(D.max(axis=1).todense()).ravel()
    amax = np.asarray(Aa.max(axis=1).todense()).ravel()
    rows = amax > 0
    assert np.all(dmax[~rows] == 0)
    return float((dmax[rows] / amax[rows]).max()) if rows.any() else 0.0
