"""Pins of the oracle's seed tree and seed management functions: the paper's
worked example, and invariants checked against the tree equation."""

import random

import pytest

from conftest import golden_lines


def _nodes(spec):
    out = []
    for item in spec:
        d, i = item.split(":")
        out.append((int(d), int(i)))
    return out


@pytest.mark.parametrize("inst", [0, 1])
def test_worked_example(O, inst):
    rows = list(golden_lines("smf_worked_example.txt"))
    D = int(rows[0][1])
    root = bytes(range(16))
    stacks = {}
    ds = []
    for i in range(1 << D):
        ds, x0 = O.SSO(inst, ds, root, D, i)
        stacks[i] = ds
        assert x0 == O.tree_node(inst, root, D, 0, i)
    for row in rows[1:]:
        if row[0] == "ds":
            i = int(row[1])
            want = _nodes(row[2:])
            assert [(n.depth, n.index) for n in stacks[i]] == want
            for n in stacks[i]:
                assert n.value == O.tree_node(inst, root, D, n.depth, n.index)
        elif row[0] == "sr":
            i, ip = int(row[1]), int(row[2])
            assert O.SR(inst, stacks[i], ip) == O.tree_node(inst, root, D, 0, ip)


@pytest.mark.parametrize("D", [1, 2, 3, 4, 5, 6])
def test_sso_sr_invariants(O, D):
    inst = D % 2
    root = bytes([D]) * 16
    leaves = [O.tree_node(inst, root, D, 0, i) for i in range(1 << D)]
    ds = []
    for i in range(1 << D):
        ds, x0 = O.SSO(inst, ds, root, D, i)
        assert x0 == leaves[i]
        assert len(ds) <= D or (i == (1 << D) - 1 and len(ds) == 1)
        for ip in range(1 << D):
            got = O.SR(inst, ds, ip)
            if ip <= i:
                assert got == leaves[ip]
            else:
                assert got is None
        # the stack is a left-to-right cover of leaves 0..i
        lo = 0
        for n in ds:
            assert n.index * (1 << n.depth) == lo
            lo = (n.index + 1) * (1 << n.depth)
        assert lo == i + 1
    # the last disclosure is the root alone
    assert [(n.depth, n.index) for n in ds] == [(D, 0)]


def test_sc_matches_tree_equation(O):
    rng = random.Random(3)
    D = 7
    root = bytes(range(16, 32))
    for _ in range(30):
        d0 = rng.randrange(0, D + 1)
        i0 = rng.randrange(0, 1 << (D - d0))
        d1 = rng.randrange(0, d0 + 1)
        i1 = (i0 << (d0 - d1)) + rng.randrange(0, 1 << (d0 - d1))
        x0 = O.tree_node(1, root, D, d0, i0)
        assert O.SC(1, x0, d0, i0, d1, i1) == O.tree_node(1, root, D, d1, i1)
    with pytest.raises(ValueError):
        O.SC(1, root, 3, 0, 1, 5)  # not a descendant


def test_ds_wire_roundtrip_and_strictness(O):
    nodes = [O.Node(2, 0, bytes(16)), O.Node(1, 2, bytes(range(16))), O.Node(0, 6, b"\xff" * 16)]
    buf = O.ds_encode(nodes)
    assert len(buf) == 1 + 24 * 3
    assert O.ds_decode(buf) == nodes
    bad = bytearray(buf)
    bad[2] = 1  # a pad byte
    with pytest.raises(ValueError):
        O.ds_decode(bytes(bad))
    with pytest.raises(ValueError):
        O.ds_decode(buf[:-1])
