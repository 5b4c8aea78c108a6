"""Front end for real workloads: Gmsh mesh files, band tables, 3D quadratures
over 2D domains.

The paper's workflow reads COMSOL or Gmsh meshes with labelled boundaries and
source regions, and band-resolved phonon properties (heat capacity, group
velocity, relaxation time) tabulated from first-principles data (Methods).
The library reads Gmsh files itself (nbte_mesh_read_gmsh: cells, tagged
boundary faces, cell regions); this module writes them (to export a mesh) and
reads band tables:

  band table file: one band per line, whitespace-separated columns
      C [J m^-3 K^-1]   v [m/s]   tau [s]
  lines starting with '#' are comments.

bin_modes reduces a spectral (per-mode) table to B bands by frequency: each
band keeps the heat capacity, the ballistic energy flux sum C v and the
kinetic conductivity sum C v^2 tau of its modes (C_b = sum C, v_b = sum C v /
C_b, tau_b = sum C v^2 tau / (C_b v_b^2)).
"""
from __future__ import annotations

import numpy as np

GMSH_TYPE = {"tri3": 2, "quad4": 3, "tet4": 4, "hex8": 5}
GMSH_FACE_TYPE = {"tri3": 1, "quad4": 1, "tet4": 2, "hex8": 3}


def write_gmsh(path, dim, xyz, cell_type, cells, bfaces, bface_tag, cell_region=None, version="4.1"):
    """Write a mesh as an ASCII Gmsh file (MSH 4.1 or 2.2): cells as elements
    of the mesh dimension with their region as physical group, boundary faces
    as elements one dimension lower with their tag as physical group.  Node
    tags are 1-based (node k of xyz has tag k + 1)."""
    xyz = np.asarray(xyz, float)
    cells = np.asarray(cells, np.int64)
    bfaces = np.asarray(bfaces, np.int64)
    tags = np.asarray(bface_tag, np.int64)
    region = np.zeros(len(cells), np.int64) if cell_region is None else np.asarray(cell_region, np.int64)
    X = np.zeros((len(xyz), 3))
    X[:, :xyz.shape[1]] = xyz
    ct, ft = GMSH_TYPE[cell_type], GMSH_FACE_TYPE[cell_type]
    lines = ["$MeshFormat", f"{version} 0 8", "$EndMeshFormat"]
    if version.startswith("2"):
        lines += ["$Nodes", str(len(X))]
        lines += [f"{k + 1} {x[0]:.17g} {x[1]:.17g} {x[2]:.17g}" for k, x in enumerate(X)]
        lines += ["$EndNodes", "$Elements", str(len(bfaces) + len(cells))]
        e = 1
        for f, t in zip(bfaces, tags):
            lines.append(f"{e} {ft} 2 {t} {t} " + " ".join(str(n + 1) for n in f))
            e += 1
        for c, r in zip(cells, region):
            lines.append(f"{e} {ct} 2 {r} {r} " + " ".join(str(n + 1) for n in c))
            e += 1
        lines.append("$EndElements")
    else:
        # one entity per physical group (faces: dim - 1, cells: dim), no bounding-entity lists
        ftags = sorted(set(tags.tolist()))
        rtags = sorted(set(region.tolist()))
        fent = {t: k + 1 for k, t in enumerate(ftags)}
        rent = {r: k + 1 for k, r in enumerate(rtags)}
        counts = [0, 0, 0, 0]
        counts[dim - 1] = len(ftags)
        counts[dim] = len(rtags)
        lines += ["$Entities", " ".join(str(c) for c in counts)]
        lo, hi = X.min(axis=0), X.max(axis=0)
        box = " ".join(f"{float(v):.17g}" for v in (*lo, *hi))
        for d in range(4):
            groups = ftags if d == dim - 1 else (rtags if d == dim else [])
            ent = fent if d == dim - 1 else rent
            for g in groups:
                lines.append(f"{ent[g]} {box} 1 {g} 0")
        lines.append("$EndEntities")
        lines += ["$Nodes", f"1 {len(X)} 1 {len(X)}", f"{dim} 1 0 {len(X)}"]
        lines += [str(k + 1) for k in range(len(X))]
        lines += [f"{x[0]:.17g} {x[1]:.17g} {x[2]:.17g}" for x in X]
        lines.append("$EndNodes")
        # element blocks follow the given order: a new block wherever the group changes
        blocks = []
        e = 1
        for d, ent, typ, items, groups in ((dim - 1, fent, ft, bfaces, tags), (dim, rent, ct, cells, region)):
            for j in range(len(items)):
                if not blocks or blocks[-1][0] != d or blocks[-1][1] != ent[int(groups[j])]:
                    blocks.append((d, ent[int(groups[j])], typ, []))
                blocks[-1][3].append(f"{e} " + " ".join(str(n + 1) for n in items[j]))
                e += 1
        lines += ["$Elements", f"{len(blocks)} {e - 1} 1 {e - 1}"]
        for d, ent, typ, body in blocks:
            lines.append(f"{d} {ent} {typ} {len(body)}")
            lines += body
        lines.append("$EndElements")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def load_band_table(path):
    """(C, v, tau) arrays of a band table file (see the module docstring)."""
    rows = []
    with open(path) as f:
        for ln, line in enumerate(f, 1):
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            parts = line.split()
            if len(parts) != 3:
                raise ValueError(f"{path}:{ln}: expected 3 columns (C v tau), got {len(parts)}")
            vals = [float(x) for x in parts]
            if not all(np.isfinite(vals)) or min(vals) <= 0:
                raise ValueError(f"{path}:{ln}: values must be finite and positive")
            rows.append(vals)
    if not rows:
        raise ValueError(f"{path}: no bands")
    a = np.array(rows)
    return a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy()


def save_band_table(path, C, v, tau, comment=""):
    with open(path, "w") as f:
        if comment:
            f.write("".join(f"# {ln}\n" for ln in comment.splitlines()))
        f.write("# C [J m^-3 K^-1]  v [m/s]  tau [s]\n")
        for c, vv, t in zip(C, v, tau):
            f.write(f"{float(c):.17g} {float(vv):.17g} {float(t):.17g}\n")


def bin_modes(freq, C, v, tau, n_bands, edges=None):
    """Reduce per-mode properties to n_bands frequency bands (equal-width bins
    over the frequency range unless edges are given).  Returns (C_b, v_b,
    tau_b, edges); every band keeps sum C, sum C v and sum C v^2 tau of its
    modes.  Empty bins are dropped."""
    freq, C, v, tau = (np.asarray(x, float) for x in (freq, C, v, tau))
    if edges is None:
        edges = np.linspace(freq.min(), freq.max(), n_bands + 1)
        edges[-1] = np.nextafter(edges[-1], np.inf)
    idx = np.clip(np.searchsorted(edges, freq, side="right") - 1, 0, len(edges) - 2)
    out = []
    for b in range(len(edges) - 1):
        m = idx == b
        if not np.any(m):
            continue
        Cb = C[m].sum()
        vb = (C[m] * v[m]).sum() / Cb
        taub = (C[m] * v[m] ** 2 * tau[m]).sum() / (Cb * vb * vb)
        out.append((Cb, vb, taub))
    a = np.array(out)
    return a[:, 0], a[:, 1], a[:, 2], edges
