"""The row partition of the P1-P1 pattern that the one-kernel-per-iteration
Poisson CG runs on (host logic, no GPU). Checked against the CSR pattern:
perm is a permutation, parts are contiguous and no larger than asked, the halo
of each part is exactly the set of columns its rows reference in other parts,
and every matrix entry is reached through the part-local column indices and
maps to its own slot of the global SELL-64 layout; parts are compact (small
halos) on structured and jittered meshes."""
import numpy as np
import pytest

from paper_2605_25403_amd import ipcs as I
from paper_2605_25403_amd.workloads import jittered_mesh


def global_sell_ptr(rp):
    n = len(rp) - 1
    lens = np.diff(rp)
    ns = (n + 63) // 64
    w = np.array([lens[64 * s:64 * s + 64].max(initial=0) for s in range(ns)], dtype=np.int64)
    return np.concatenate([[0], np.cumsum(64 * w)])


def check_partition(m, rows_max):
    rp, col = I.ipcs_mesh_pattern(m.h, I.IPCS_PATTERN_P1P1)
    n = len(rp) - 1
    P = I.ipcs_mesh_p1_partition(m.h, rows_max)
    perm, pptr, hptr, halo = P["perm"], P["part_ptr"], P["halo_ptr"], P["halo"]
    np.testing.assert_array_equal(np.sort(perm), np.arange(n))
    iperm = np.empty(n, np.int64)
    iperm[perm] = np.arange(n)
    sizes = np.diff(pptr)
    assert pptr[0] == 0 and pptr[-1] == n and sizes.min() > 0 and sizes.max() <= rows_max
    assert len(sizes) >= -(-n // rows_max)
    gsp = global_sell_ptr(rp)
    sptr, sl_ptr, lcol, src = P["sptr"], P["slice_ptr"], P["lcol"], P["src"]
    lds = 0
    for p in range(len(sizes)):
        p0, p1 = pptr[p], pptr[p + 1]
        own = p1 - p0
        assert np.all(np.diff(perm[p0:p1]) > 0)          # original order kept in a part
        rows = perm[p0:p1]
        cols = np.concatenate([iperm[col[rp[o]:rp[o + 1]]] for o in rows])
        ext = np.unique(cols[(cols < p0) | (cols >= p1)])
        h = halo[hptr[p]:hptr[p + 1]]
        np.testing.assert_array_equal(h, ext)
        lds = max(lds, own + len(h))
        local_to_po = np.concatenate([np.arange(p0, p1), h])
        assert sl_ptr[p + 1] - sl_ptr[p] == -(-own // 64)
        for j in range(sl_ptr[p + 1] - sl_ptr[p]):
            s = sl_ptr[p] + j
            w = (sptr[s + 1] - sptr[s]) // 64
            for q in range(64):
                l = 64 * j + q
                e = sptr[s] + 64 * np.arange(w) + q
                if l >= own:
                    assert np.all(src[e] == -1)
                    continue
                o = perm[p0 + l]
                ln = rp[o + 1] - rp[o]
                assert ln <= w
                got = perm[local_to_po[lcol[e[:ln]]]]
                np.testing.assert_array_equal(got, col[rp[o]:rp[o + 1]])
                np.testing.assert_array_equal(src[e[:ln]], gsp[o >> 6] + 64 * np.arange(ln) + (o & 63))
                assert np.all(src[e[ln:]] == -1)
                assert np.all(lcol[e[ln:]] == lcol[e[ln - 1]])
    assert lds == P["lds_rows"]
    return P, n


@pytest.mark.parametrize("dim,n,rows", [(2, 1, 64), (2, 5, 64), (2, 23, 128), (2, 40, 1024),
                                        (3, 2, 64), (3, 6, 256)])
def test_structured_partitions(dim, n, rows):
    m = I.Mesh.unit_square(n) if dim == 2 else I.Mesh.unit_cube(n)
    check_partition(m, rows)


@pytest.mark.parametrize("dim,n,seed,rows", [(2, 21, 4, 128), (3, 5, 1, 128)])
def test_jittered_partitions(dim, n, seed, rows):
    m = I.Mesh.from_arrays(*jittered_mesh(dim, n, seed))
    check_partition(m, rows)


def test_parts_are_compact():
    """On a structured square the parts are patches: the halo is a perimeter,
    about 4 sqrt(rows) per part, not a band of whole grid lines."""
    m = I.Mesh.unit_square(128)
    P = I.ipcs_mesh_p1_partition(m.h, 1024)
    nparts = len(P["part_ptr"]) - 1
    per_part = len(P["halo"]) / nparts
    assert per_part <= 5 * np.sqrt(1024), per_part
    # a relabelled mesh partitions by coordinates, not by labels
    j = I.Mesh.from_arrays(*jittered_mesh(2, 128, 3))
    Pj = I.ipcs_mesh_p1_partition(j.h, 1024)
    assert len(Pj["halo"]) / (len(Pj["part_ptr"]) - 1) <= 6 * np.sqrt(1024)


def test_partition_arguments():
    m = I.Mesh.unit_square(4)
    with pytest.raises(I.IpcsError):
        I.ipcs_mesh_p1_partition(m.h, 32)
    with pytest.raises(I.IpcsError):
        I.ipcs_mesh_p1_partition(m.h, 4096)
    with pytest.raises(I.IpcsError):
        I.ipcs_run_workspace_bytes(m.h, I.ipcs_params_default(poisson_part_rows=7))
