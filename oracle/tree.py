"""Hierarchical factorization of the primitives — test oracle.

Written from Sec. 4 (Optimizations) of the paper:

  * the machine is a vector of integer factors of p, the first factor being
    the highest level (Sec. 4.2);
  * consecutive ranks fill the innermost groups: ranks whose ids share
    ``r // B_k`` are in one depth-k group, with ``B_k`` the product of the
    factors below level k (same section);
  * a multicast is routed down the tree: at each level the current root sends
    one copy into every sibling group that holds a leaf, to a staging rank of
    that group, which then acts as the root inside its group; the tree is
    pruned to the groups that hold leaves (same section, and the worked
    {2,2,3} broadcast of Sec. 4.3);
  * a reduction is the mirror image: partial results are formed bottom-up at
    one staging rank per group and travel up one level at a time;
  * striping splits a primitive into s branches owned by s ranks of the
    root's group: an intra-group scatter, a fence, then one multicast per
    stripe from its owner (Sec. 4.3); for a reduction the
    mirror (per-stripe reduction into the owner, fence, owner to root);
  * pipelining splits every branch into m channels; it changes neither which
    ranks exchange data nor the order in which operands are combined, so it
    does not appear here (Sec. 4.5).

Readings where the paper is silent (each listed in the design notes):
  * staging rank of a group = the rank at the current root's offset inside
    the group if that rank is a leaf, else the lowest leaf of the group; for
    a reduction, the group that contains the root is hosted by the root;
  * stripe group = the root's smallest enclosing group whose size is at least
    s and divisible by s; stripe t is owned by the rank at the root's offset
    plus t * (size / s), modulo the group size; only primitives with a leaf
    outside the stripe group are striped;
  * a striped multicast's branches do not send back to the root (which
    already holds the data) — the root gets one local copy if it is a leaf
    and its send and receive buffers differ;
  * a group with a single contributing child forms no reduction node: the
    child's value is read where it lies;
  * a reduction node combines its operands in ascending child-group order,
    left to right (the paper fixes no order; this one is what the
    order-exact expectations below assume).

Also here: the minimum bytes that must cross the top level for each
collective, derived from Table 3 (per-node
bound times the number of nodes).

Parity: pinned by tests/test_oracle_tree.py against the worked examples of
Sec. 4.3 (golden hop list), Fig. 1 (3 versus 1 cross-node copies), the striped four-stage
tree, closed forms for hop counts per level, and brute-force minima.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------- groups
def block_sizes(h: list[int]) -> list[int]:
    """``B[k]`` = ranks per depth-k group; ``B[0]`` = p, ``B[len(h)]`` = 1."""
    p = int(np.prod(h)) if h else 1
    out = [p]
    for f in h:
        out.append(out[-1] // f)
    return out


def depth(a: int, b: int, h: list[int]) -> int:
    """Level of the hop a -> b: the first depth (1 = highest) whose groups separate a and b; 0 if a == b."""
    if a == b:
        return 0
    B = block_sizes(h)
    for k in range(1, len(h) + 1):
        if a // B[k] != b // B[k]:
            return k
    raise AssertionError("unreachable")


def group_of(r: int, k: int, h: list[int]) -> tuple[int, int]:
    """(first rank, size) of rank r's depth-k group."""
    B = block_sizes(h)
    return (r // B[k]) * B[k], B[k]


# ------------------------------------------------------------- multicast
@dataclass
class Hop:
    src: int
    dst: int
    depth: int
    stage: int
    stripe: int = 0


def multicast_hops(root: int, leaves, h: list[int], stage0: int = 0, stripe: int = 0) -> list[Hop]:
    """Hops of the tree factorization of M(root, leaves), excluding a local copy at the root.

    Each hop's ``stage`` is one more than the stage at which its sender
    obtained the data (the root holds it before ``stage0``).
    """
    B = block_sizes(h)
    L = len(h)
    hops: list[Hop] = []

    def rec(src: int, lv: set, lo: int, k: int, st: int):
        # src lies in the depth-(k-1) group starting at lo; split it into its f_k subgroups
        if k > L or not lv:
            return
        sub = B[k]
        mine = (src - lo) // sub
        for c in range(h[k - 1]):
            clo = lo + c * sub
            cl = {x for x in lv if clo <= x < clo + sub}
            if c == mine:
                rec(src, cl - {src}, clo, k + 1, st)
            elif cl:
                same = clo + (src - lo) % sub
                stg = same if same in cl else min(cl)
                hops.append(Hop(src, stg, k, st, stripe))
                rec(stg, cl - {stg}, clo, k + 1, st + 1)

    rec(root, set(leaves) - {root}, 0, 1, stage0)
    return hops


# ------------------------------------------------------------- reduction
@dataclass
class Node:
    host: int
    depth: int                      # level of the group this node reduces (1 = whole machine)
    children: list = field(default_factory=list)   # Node or int (a leaf rank)


def reduction_tree(leaves, root: int, h: list[int]):
    """Tree of R(leaves, root): a Node, or a leaf rank when only one leaf contributes."""
    B = block_sizes(h)
    L = len(h)
    lvset = set(leaves)

    def host_of(lo: int, size: int) -> int:
        if lo <= root < lo + size:
            return root
        same = lo + root % size
        if same in lvset:
            return same
        return min(x for x in lvset if lo <= x < lo + size)

    def rec(lo: int, k: int):
        size = B[k - 1]
        inside = [x for x in lvset if lo <= x < lo + size]
        if not inside:
            return None
        if size == 1:
            return lo
        sub = B[k]
        kids = []
        for c in range(h[k - 1]):
            t = rec(lo + c * sub, k + 1)
            if t is not None:
                kids.append(t)
        if len(kids) == 1:
            return kids[0]
        return Node(host_of(lo, size), k, kids)

    if not lvset:
        return None
    if L == 0:
        return min(lvset)
    return rec(0, 1)


def host(t) -> int:
    return t if isinstance(t, int) else t.host


def reduction_nodes(tree) -> list[Node]:
    """All nodes of a reduction tree, children before parents."""
    out = []

    def rec(t):
        if isinstance(t, Node):
            for c in t.children:
                rec(c)
            out.append(t)

    rec(tree)
    return out


def tree_depth_stages(tree) -> int:
    """Number of dependent reduction stages on the longest path (0 for a bare leaf)."""
    if not isinstance(tree, Node):
        return 0
    return 1 + max(tree_depth_stages(c) for c in tree.children)


# ------------------------------------------------------------- striping
def stripe_owners(root: int, leaves, h: list[int], s: int):
    """Owners of the s stripes of a primitive rooted at ``root``, or None when it is not striped."""
    if s <= 1:
        return None
    B = block_sizes(h)
    for k in range(len(h), -1, -1):
        size = B[k]
        if size >= s and size % s == 0:
            lo = (root // size) * size
            if all(lo <= x < lo + size for x in leaves):
                return None
            step = size // s
            return [lo + ((root - lo) + t * step) % size for t in range(s)]
    raise ValueError("stripe factor does not divide any group")


def split(n: int, parts: int, align: int) -> list[tuple[int, int]]:
    """Contiguous (offset, length) pieces of n elements, boundaries on multiples of ``align``.

    Whole ``align`` units are spread as evenly as possible (earlier pieces get
    the extra unit); the last piece also takes the remainder below ``align``.
    """
    units, rem = divmod(n, align)
    out = []
    off = 0
    for t in range(parts):
        u = units // parts + (1 if t < units % parts else 0)
        ln = u * align + (rem if t == parts - 1 else 0)
        out.append((off, ln))
        off += ln
    return out


# ------------------------------------------------------------ accounting
def prim_transfers(kind: str, root: int, leaves, n: int, h: list[int], s: int = 1,
                   align: int = 1, self_copy: bool = True):
    """Logical transfers (src, dst, elements) of one factorized primitive.

    ``kind`` is "M" or "R". A reduction node contributes one transfer per
    child hosted on another rank; a local copy (src == dst) is listed when
    the root is a multicast leaf with distinct buffers (``self_copy``).
    """
    leaves = list(leaves)
    out = []
    if kind == "M":
        owners = stripe_owners(root, leaves, h, s)
        if owners is None:
            for hp in multicast_hops(root, leaves, h):
                out.append((hp.src, hp.dst, n))
        else:
            for t, (off, ln) in enumerate(split(n, s, align)):
                if ln == 0:
                    continue
                o = owners[t]
                if o != root:
                    out.append((root, o, ln))
                for hp in multicast_hops(o, set(leaves) - {o, root}, h):
                    out.append((hp.src, hp.dst, ln))
        if root in leaves and self_copy:
            out.append((root, root, n))
        return out
    owners = stripe_owners(root, leaves, h, s)
    pieces = [(root, n)] if owners is None else [
        (owners[t], ln) for t, (off, ln) in enumerate(split(n, s, align)) if ln > 0]
    for own, ln in pieces:
        tree = reduction_tree(leaves, own, h)
        if isinstance(tree, int):
            out.append((tree, own, ln))
        else:
            for nd in reduction_nodes(tree):
                for c in nd.children:
                    out.append((host(c), nd.host, ln))
            if tree.host != own:
                out.append((tree.host, own, ln))
        if own != root:
            out.append((own, root, ln))
    return out


def level_bytes(transfers, acct: list[int], esize: int) -> list[int]:
    """Bytes per depth of an accounting hierarchy; index 0 = local (same rank)."""
    out = [0] * (len(acct) + 1)
    for a, b, n in transfers:
        out[depth(a, b, acct)] += n * esize
    return out


# collective -> list of (kind, root, leaves, count) in units of d, p, for s = 1
def collective_prims(name: str, p: int, d: int, root: int = 0):
    U = list(range(p))
    if name == "broadcast":
        return [("M", root, U, d * p)]
    if name == "reduce":
        return [("R", root, U, d * p)]
    if name == "all_gather":
        return [("M", i, U, d) for i in U]
    if name == "reduce_scatter":
        return [("R", j, U, d) for j in U]
    if name == "all_reduce":
        return [("R", j, U, d) for j in U] + [("M", i, [r for r in U if r != i], d) for i in U]
    if name == "scatter":
        return [("M", root, [j], d) for j in U]
    if name == "gather":
        return [("M", i, [root], d) for i in U]
    if name == "all_to_all":
        return [("M", i, [j], d) for i in U for j in U]
    raise ValueError(name)


def collective_level_bytes(name: str, h: list[int], d: int, acct: list[int] | None = None,
                           s: int = 1, esize: int = 1, align: int = 1, root: int = 0) -> list[int]:
    """Per-depth logical bytes of a collective factorized on ``h`` and counted on ``acct``."""
    p = int(np.prod(h))
    acct = h if acct is None else acct
    tr = []
    for kind, r, lv, n in collective_prims(name, p, d, root):
        tr += prim_transfers(kind, r, lv, n, h, s, align)
    return level_bytes(tr, acct, esize)


def min_top_bytes(name: str, p: int, g: int, d: int) -> int:
    """Least data that must cross the top level (in elements of d), for f_1 = p / g nodes.

    Derived from Table 3: its bound is the
    per-node volume at rate k*f, and every node must receive that volume
    through its own links. With n_1 = p/g nodes and buffers of d*p:
      Broadcast / Reduce : each non-root node receives one full buffer
      Gather / Scatter   : the root node exchanges d with each outside rank
      All-Gather / Reduce-Scatter : each node receives (p - g) chunks
      All-Reduce         : twice the All-Gather volume (scatter + gather halves)
      All-to-All         : each of the g ranks of a node receives (p - g) chunks
    """
    n1 = p // g
    if name in ("broadcast", "reduce"):
        return (n1 - 1) * d * p
    if name in ("gather", "scatter"):
        return (p - g) * d
    if name in ("all_gather", "reduce_scatter"):
        return n1 * (p - g) * d
    if name == "all_reduce":
        return 2 * n1 * (p - g) * d
    if name == "all_to_all":
        return p * (p - g) * d
    raise ValueError(name)


# --------------------------------------------------- order-exact reduction values
def tree_reduce(values: dict, leaves, root: int, h: list[int], combine) -> np.ndarray:
    """Evaluate R(leaves, root) by its factorized tree with a caller-given node operation.

    ``values[r]`` is leaf r's operand; ``combine(list_of_operands)`` forms
    one node's output from its operands in ascending child order (for
    instance a left-to-right float32 sum, or a dequantize / sum / requantize
    step). A single-leaf tree returns the leaf's operand unchanged.
    """
    tree = reduction_tree(leaves, root, h)

    def ev(t):
        if isinstance(t, int):
            return values[t]
        return combine([ev(c) for c in t.children])

    return ev(tree)


def striped_reduce(values: dict, leaves, root: int, n: int, h: list[int], s: int, align: int,
                   combine) -> np.ndarray:
    """R(leaves, root) over n elements with striping: each stripe follows the tree of its owner."""
    owners = stripe_owners(root, leaves, h, s)
    if owners is None:
        return tree_reduce(values, leaves, root, h, combine)
    parts = []
    for t, (off, ln) in enumerate(split(n, s, align)):
        sub = {r: v[off:off + ln] for r, v in values.items()}
        parts.append(tree_reduce(sub, leaves, owners[t], h, combine))
    return np.concatenate(parts)


def sum_f32(ops: list[np.ndarray]) -> np.ndarray:
    """float32 left-to-right sum, rounding after every addition (IEEE round-to-nearest-even)."""
    acc = np.asarray(ops[0], dtype=np.float32).copy()
    for v in ops[1:]:
        acc = (acc + np.asarray(v, dtype=np.float32)).astype(np.float32)
    return acc


# ------------------------------------------------------------- hybrid ring + tree
def ring_depth(h: list[int], n: int) -> int:
    """Depth k whose groups are the ring's conceptual nodes (p/n ranks each), or raise."""
    B = block_sizes(h)
    p = B[0]
    if n < 1 or p % n:
        raise ValueError("ring length must divide p")
    for k in range(len(B)):
        if B[k] == p // n:
            return k
    raise ValueError("p / ring must be a group size of the hierarchy")


def ring_chain(root: int, leaves, h: list[int], n: int) -> list[int]:
    """First ranks of the conceptual nodes the ring visits after the root's, in ring order (Sec. 4.4):
    the next node, the one after, ... skipping nodes without a leaf."""
    k = ring_depth(h, n)
    size = block_sizes(h)[k]
    mine = root // size
    out = []
    for c in range(1, n):
        node = (mine + c) % n
        lo = node * size
        if any(lo <= x < lo + size for x in leaves):
            out.append(lo)
    return out


def ring_multicast_hops(root: int, leaves, h: list[int], n: int, s: int = 1, align: int = 1, count: int = None):
    """Hops of a multicast under ring(n) and stripe(s): striping, then the ring, then trees (Sec. 4.4).

    Returns (hops, nstages): each hop carries (src, dst, depth, stage, stripe, ring_step). Stage 0 is the
    intra-node scatter, ring hops follow one stage per node, and every node's inner tree starts when
    its holder has the stripe."""
    leaves = set(leaves)
    k = ring_depth(h, n)
    size = block_sizes(h)[k]
    inner = h[k:]
    if s > 1:
        own = stripe_owners(root, [x for x in leaves], h, s)
    else:
        own = None
    if own is None:
        own = [root]
    hops = []

    def inner_tree(src, lv, lo, stage, stripe):
        # the tree inside one conceptual node, on the inner hierarchy
        loc = [x - lo for x in lv]
        for hp in multicast_hops(src - lo, loc, inner, stage0=stage, stripe=stripe):
            hops.append(Hop(hp.src + lo, hp.dst + lo, depth(hp.src + lo, hp.dst + lo, h), hp.stage, stripe))

    chain = ring_chain(root, leaves, h, n)
    for t, o in enumerate(own):
        st = 0
        if o != root:
            hops.append(Hop(root, o, depth(root, o, h), 0, t))
            st = 1
        off = o % size
        lo0 = (root // size) * size
        inner_tree(o, [x for x in leaves if lo0 <= x < lo0 + size and x not in (o, root)], lo0, st, t)
        prev, pst = o, st
        for c, lo in enumerate(chain):
            dst = lo + off
            hops.append(Hop(prev, dst, depth(prev, dst, h), pst, t))
            inner_tree(dst, [x for x in leaves if lo <= x < lo + size and x != dst], lo, pst + 1, t)
            prev, pst = dst, pst + 1
    nst = 1 + max(hp.stage for hp in hops) if hops else 0
    return hops, nst


def ring_reduce(values: dict, leaves, root: int, h: list[int], n: int, combine):
    """R(leaves, root) under ring(n) without striping: each conceptual node reduces its own leaves by its
    inner tree; the top node of a node's tree also takes the partial arriving from the next node of the
    ring, as its last operand; the root's node finishes the sum. ``values[r]`` are leaf operands."""
    k = ring_depth(h, n)
    size = block_sizes(h)[k]
    inner = h[k:]
    leaves = sorted(set(leaves))
    chain = ring_chain(root, leaves, h, n)
    off = root % size

    def node_value(lo, holder, incoming):
        lv = [x - lo for x in leaves if lo <= x < lo + size]
        if not lv:
            return incoming
        tree = reduction_tree(lv, holder - lo, inner)

        def ev(t, top):
            if isinstance(t, int):
                v = values[t + lo]
                return v if not (top and incoming is not None) else combine([v, incoming])
            ops = [ev(c, False) for c in t.children]
            if top and incoming is not None:
                ops.append(incoming)
            return combine(ops)

        return ev(tree, True)

    incoming = None
    for lo in reversed(chain):
        incoming = node_value(lo, lo + off, incoming)
    lo0 = (root // size) * size
    return node_value(lo0, root, incoming)
