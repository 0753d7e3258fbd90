"""Mesh variants for tests (built from the seeded generator's meshes)."""
import numpy as np

import gks_inputs as gi


def split_some_triangles(mesh, every=7):
    """The mesh with every `every`-th triangle split at its centroid into
    three: the three new cells are mutually adjacent (a 3-cycle of the cell
    graph).  Non-periodic meshes only."""
    xy = [mesh.xy]
    tri, tag = [], []
    nv = mesh.xy.shape[0]
    for t in range(mesh.tri.shape[0]):
        a, b, c = mesh.tri[t]
        ta, tb, tc = mesh.edge_tag[t]
        if t % every:
            tri.append((a, b, c))
            tag.append((ta, tb, tc))
            continue
        xy.append(mesh.xy[[a, b, c]].mean(axis=0)[None, :])
        p = nv
        nv += 1
        tri += [(a, b, p), (b, c, p), (c, a, p)]
        tag += [(ta, 0, 0), (tb, 0, 0), (tc, 0, 0)]
    return gi.Mesh(xy=np.concatenate(xy), tri=np.array(tri, dtype=np.int32), edge_tag=np.array(tag, dtype=np.int32),
                   periodic=mesh.periodic, L=mesh.L, origin=mesh.origin, bc_table=mesh.bc_table)
