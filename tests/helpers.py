"""Conversions between the oracle's dense tensors and the library's layouts.

Test infrastructure only.  The oracle keeps dense arrays with a (N, 2Sz)
label per bond state (sorted by label); the library uses the layouts
documented in include/dmrg.h (fine blocks for site tensors, merged sectors
for two-site vectors).  Nothing here does any of the method's arithmetic.
"""

from __future__ import annotations

import numpy as np

SITE_QN = [(0, 0), (1, 1), (1, -1), (2, 0)]
SYS_ORDER = [3, 1, 2, 0]


def sectors(labels):
    """Sorted [(N, 2Sz, dim)] of a label array (m, 2)."""
    out = {}
    for n, s in np.asarray(labels).reshape(-1, 2):
        out[(int(n), int(s))] = out.get((int(n), int(s)), 0) + 1
    return [(q[0], q[1], d) for q, d in sorted(out.items())]


def _rows_of(labels, q):
    return np.nonzero(np.all(np.asarray(labels) == q, axis=1))[0]


def site_fine_blocks(T, lab_l, lab_r):
    """Dense site tensor (m_l, 4, m_r) -> flat fine-block values."""
    out = []
    for n, s2, _ in sectors(lab_l):
        rows = _rows_of(lab_l, (n, s2))
        for s in range(4):
            qr = (n + SITE_QN[s][0], s2 + SITE_QN[s][1])
            cols = _rows_of(lab_r, qr)
            if len(cols) == 0:
                continue
            out.append(T[np.ix_(rows, [s], cols)][:, 0, :].ravel())
    return np.concatenate(out) if out else np.zeros(0)


def two_site_sectors(lab_l, lab_r):
    """Middle sectors q with nonempty sys and env spaces, sorted."""
    ql = {tuple(x) for x in np.asarray(lab_l).reshape(-1, 2)}
    qr = {tuple(x) for x in np.asarray(lab_r).reshape(-1, 2)}
    cand = sorted({(a + SITE_QN[s][0], b + SITE_QN[s][1]) for a, b in ql for s in range(4)})
    out = []
    for q in cand:
        sys_ok = any((q[0] - SITE_QN[s][0], q[1] - SITE_QN[s][1]) in ql for s in range(4))
        env_ok = any((q[0] + SITE_QN[t][0], q[1] + SITE_QN[t][1]) in qr for t in range(4))
        if sys_ok and env_ok:
            out.append(q)
    return out


def merged_index(lab_l, lab_r):
    """Flat positions of the merged layout inside the dense (m_l,4,4,m_r) array."""
    lab_l, lab_r = np.asarray(lab_l), np.asarray(lab_r)
    ml, mr = len(lab_l), len(lab_r)
    idx = []
    for q in two_site_sectors(lab_l, lab_r):
        rows = []  # (a, s) in order of Q_l ascending (a ascending)
        for a in range(ml):
            for s in range(4):
                if (lab_l[a][0] + SITE_QN[s][0], lab_l[a][1] + SITE_QN[s][1]) == q:
                    rows.append((a, s))
        cols = []  # (t, b), t-major
        for t in range(4):
            for b in range(mr):
                if (lab_r[b][0] - SITE_QN[t][0], lab_r[b][1] - SITE_QN[t][1]) == q:
                    cols.append((t, b))
        for a, s in rows:
            for t, b in cols:
                idx.append(((a * 4 + s) * 4 + t) * mr + b)
    return np.array(idx, dtype=np.int64), (ml, 4, 4, mr)


def dense_to_merged(psi, lab_l, lab_r):
    idx, shape = merged_index(lab_l, lab_r)
    return np.asarray(psi).reshape(-1)[idx]


def merged_to_dense(vec, lab_l, lab_r):
    idx, shape = merged_index(lab_l, lab_r)
    out = np.zeros(int(np.prod(shape)))
    out[idx] = vec
    return out.reshape(shape)


# --- environment operators in the channel-major block format of dmrg_env_import ----

def env_block_shapes(sectors_list, shifts):
    """Per channel the blocks (Q + dq <- Q) of a bond with sectors
    [(N, 2Sz, dim)] (sorted): list over channels of [(out, in, rows, cols)]
    with sector indices, in the documented order."""
    idx = {(n, s): i for i, (n, s, _) in enumerate(sectors_list)}
    out = []
    for dq in shifts:
        blocks = []
        for i, (n, s, d) in enumerate(sectors_list):
            o = idx.get((n + dq[0], s + dq[1]))
            if o is not None:
                blocks.append((o, i, sectors_list[o][2], d))
        out.append(blocks)
    return out


def env_blocks_to_dense(values, sectors_list, shifts):
    """Block values -> dense (D, m, m) with states in sector order."""
    offs = np.cumsum([0] + [d for _, _, d in sectors_list])
    m = int(offs[-1])
    dense = np.zeros((len(shifts), m, m))
    pos = 0
    for x, blocks in enumerate(env_block_shapes(sectors_list, shifts)):
        for o, i, r, c in blocks:
            dense[x, offs[o]:offs[o] + r, offs[i]:offs[i] + c] = np.asarray(values[pos:pos + r * c]).reshape(r, c)
            pos += r * c
    assert pos == len(values)
    return dense


def env_values_to_blocks(values, sectors_list, shifts):
    """Channel-major block values -> per channel {(Q_out, Q_in): block view}
    (no copies: large environments stay one array)."""
    secs = [(n, s) for n, s, _ in sectors_list]
    out, pos = [], 0
    for blocks in env_block_shapes(sectors_list, shifts):
        d = {}
        for o, i, r, c in blocks:
            d[(secs[o], secs[i])] = values[pos:pos + r * c].reshape(r, c)
            pos += r * c
        out.append(d)
    assert pos == len(values)
    return out


def merged_blocks(vec, left, right):
    """Two-site vector in the merged sector layout -> {(Q_l, s, t, Q_r): block
    view}; left, right: {(N, 2Sz): dim} of bonds j and j+2 (the layout of
    include/dmrg.h: sectors sorted, rows (Q_l, s) by Q_l, columns (t, Q_r) by t)."""
    def add(a, b, sg=1):
        return (a[0] + sg * b[0], a[1] + sg * b[1])
    cand = sorted({add(Q, SITE_QN[s]) for Q in left for s in range(4)})
    out, pos = {}, 0
    for q in cand:
        rows = [(s, add(q, SITE_QN[s], -1)) for s in SYS_ORDER if add(q, SITE_QN[s], -1) in left]
        cols = [(t, add(q, SITE_QN[t])) for t in range(4) if add(q, SITE_QN[t]) in right]
        if not rows or not cols:
            continue
        nr = sum(left[Q] for _, Q in rows)
        nc = sum(right[Q] for _, Q in cols)
        mat = vec[pos:pos + nr * nc].reshape(nr, nc)
        r0 = 0
        for s, Ql in rows:
            c0 = 0
            for t, Qr in cols:
                out[(Ql, s, t, Qr)] = mat[r0:r0 + left[Ql], c0:c0 + right[Qr]]
                c0 += right[Qr]
            r0 += left[Ql]
        pos += nr * nc
    assert pos == len(vec)
    return out


def site_value_count(bonds):
    """Values of the fine-block site tensors of bonds [{(N, 2Sz): dim}]."""
    n = 0
    for j in range(len(bonds) - 1):
        for Q, m in bonds[j].items():
            for s in range(4):
                n += m * bonds[j + 1].get((Q[0] + SITE_QN[s][0], Q[1] + SITE_QN[s][1]), 0)
    return n


# --- MPS checkpoint files (the layout documented with dmrg_mps_save) ------------------

MPS_MAGIC = b"DMRGMPS\x01"


def write_mps_file(path, K, N, two_sz, center, bonds, site_values, psi):
    """bonds: per k a list of (N, 2Sz, dim); site_values, psi: flat FP64."""
    import struct
    with open(path, "wb") as f:
        f.write(MPS_MAGIC)
        f.write(struct.pack("<4i", K, N, two_sz, center))
        for b in bonds:
            f.write(struct.pack("<i", len(b)))
            for t in b:
                f.write(struct.pack("<3i", *t))
        sv = np.ascontiguousarray(site_values, dtype="<f8")
        f.write(struct.pack("<q", sv.size))
        f.write(sv.tobytes())
        pv = np.ascontiguousarray(psi, dtype="<f8")
        f.write(struct.pack("<q", pv.size))
        f.write(pv.tobytes())


def read_mps_file(path):
    import struct
    with open(path, "rb") as f:
        data = f.read()
    assert data[:8] == MPS_MAGIC
    pos = 8
    K, N, tsz, center = struct.unpack_from("<4i", data, pos)
    pos += 16
    bonds = []
    for _ in range(K + 1):
        (n,) = struct.unpack_from("<i", data, pos)
        pos += 4
        bonds.append([tuple(struct.unpack_from("<3i", data, pos + 12 * i)) for i in range(n)])
        pos += 12 * n
    (ns,) = struct.unpack_from("<q", data, pos)
    pos += 8
    sites = np.frombuffer(data, dtype="<f8", count=ns, offset=pos).copy()
    pos += 8 * ns
    (npsi,) = struct.unpack_from("<q", data, pos)
    pos += 8
    psi = np.frombuffer(data, dtype="<f8", count=npsi, offset=pos).copy()
    pos += 8 * npsi
    assert pos == len(data)
    return dict(K=K, N=N, two_sz=tsz, center=center, bonds=bonds, sites=sites, psi=psi)
