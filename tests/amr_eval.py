"""Evaluation helpers of the adaptive runs (test infrastructure): states on
different adaptive meshes are compared on one uniform level."""
import numpy as np


def restrict_to_level(mesh_levels, mesh_G, interior, N, trees, level):
    """Conserved state on the uniform grid of `level` (host, float64):
    blocks finer than `level` are averaged (exact means of their cells),
    coarser blocks are copied into every covered cell.  interior: [nb][nvar]
    [N][N][N] (index order k, j, i); returns [nvar][nz][ny][nx]."""
    nb, nvar = interior.shape[:2]
    n = [t * N << level for t in trees]
    out = np.zeros((nvar, n[2], n[1], n[0]))
    for b in range(nb):
        lb = int(mesh_levels[b])
        u = np.asarray(interior[b], dtype=np.float64)
        if lb >= level:
            f = 1 << (lb - level)
            m = N // f
            c = u.reshape(nvar, m, f, m, f, m, f).mean(axis=(2, 4, 6))
            o = [int(mesh_G[b][a]) * N // f for a in range(3)]
            out[:, o[2]:o[2] + m, o[1]:o[1] + m, o[0]:o[0] + m] = c
        else:
            f = 1 << (level - lb)
            c = u.repeat(f, axis=1).repeat(f, axis=2).repeat(f, axis=3)
            o = [int(mesh_G[b][a]) * N * f for a in range(3)]
            out[:, o[2]:o[2] + N * f, o[1]:o[1] + N * f, o[0]:o[0] + N * f] = c
    return out


def oracle_adaptive_run(w, steps, regrid_every, log=None):
    """The adaptive run of workload w in the FP64 oracle with the paper's
    criterion: geometric initial refinement, then `steps` steps with a
    regrid after every `regrid_every` steps.  log(steps_done, oracle_mesh),
    if given, is called after each regrid and at the end.  Returns the
    oracle mesh."""
    from oracle import OracleMesh
    om = OracleMesh(w["ndim"], w["trees"], w["N"], w["g"], w["tree_size"], level=w.get("level", 0),
                    gamma=w["gamma"], cfl=w["cfl"])
    lmax = w["max_level"]
    om.set_interior_from_field(w["field"])
    for _ in range(lmax):
        lev = np.array([l for l, _ in om.forest.leaves])
        G = np.array([g for _, g in om.forest.leaves])
        if om.regrid(w["init_flags"](lev, G), 0, lmax) is None:
            break
        om.set_interior_from_field(w["field"])
    done = 0
    while done < steps:
        k = min(regrid_every, steps - done)
        om.step(k)
        done += k
        if done < steps:
            om.ghost_fill()
            om.regrid(om.lohner_flags(), 0, lmax)
        if log:
            log(done, om)
    return om
