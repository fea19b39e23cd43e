"""Reference networks and LoLa schedules (the oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Three things live here, all written from the paper's text:

1. Plaintext integer networks (exact Python integers, then mod t):
   - dense64: y = (W x)^2 for a 64-vector and a 64x64 matrix;
   - mnist:   5x5 stride-2 convolution with 5 maps -> square -> dense 845->100
              -> square -> dense 100->10 (Sec. 4.3, the network of Table 1), with
              integer biases;
   - head:    dense 4096->256 -> square -> dense 256->10 (the private head on
              deep features of Sec. 5, with a hidden layer).
2. Schedules: the paper's vector representations and matrix-vector recipes
   (Sec. 4.2) written out as op lists on ciphertext registers:
     ("mul_scalar", dst, src, w)      message times scalar (Sec. 4.2.2, conv)
     ("add", dst, a, b)
     ("add_plain", dst, src, slots)   slots: {slot index: value}
     ("mul_plain", dst, src, slots)
     ("rotate", dst, src, step)       step > 0 left, < 0 right, "row_swap"
     ("rotate_hoisted", dst, src, step)  the same rotation, digits taken before
                                      the automorphism (bfv.rotate_hoisted)
     ("square", dst, src)             ct x ct product then relinearisation
   Registers 0..n_inputs-1 hold the inputs; the schedule's "outputs" names the
   result registers.
3. Two interpreters for a schedule: on plain slot vectors mod t (every slot,
   including the ones that hold partial sums) and on ciphertexts through the
   oracle's BFV operations.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Sequence

import numpy as np

from . import bfv

ROW_SWAP = bfv.ROW_SWAP


# ---------------------------------------------------------------- plain nets
def _mod(a, t):
    return np.array([int(v) % t for v in np.asarray(a, dtype=object).ravel()],
                    dtype=np.int64).reshape(np.shape(a))


def dense64_plain(x, W):
    """Exact integers: ((W x)_j)^2."""
    y = np.asarray(W, dtype=object).dot(np.asarray(x, dtype=object))
    return y * y


# Padding of the 28x28 image to 29x29: one zero row at the bottom and one zero
# column at the right, so that 13 windows of 5 at stride 2 cover it
# (rows 2y..2y+4, y < 13).
MNIST_PAD = 29
MNIST_OUT = 13


def mnist_padded(img):
    p = np.zeros((MNIST_PAD, MNIST_PAD), dtype=np.int64)
    p[:28, :28] = img
    return p


def mnist_plain(img, wts):
    """Exact integer logits of the MNIST-shaped network."""
    p = mnist_padded(img).astype(object)
    conv = np.zeros((5, MNIST_OUT, MNIST_OUT), dtype=object)
    for m in range(5):
        for y in range(MNIST_OUT):
            for x in range(MNIST_OUT):
                win = p[2 * y:2 * y + 5, 2 * x:2 * x + 5]
                conv[m, y, x] = int((win * wts.conv_w[m].astype(object)).sum()) + int(wts.conv_b[m])
    a1 = (conv * conv).reshape(845)                       # index 169 m + 13 y + x
    h = wts.w1.astype(object).dot(a1) + wts.b1.astype(object)
    a2 = h * h
    return wts.w2.astype(object).dot(a2) + wts.b2.astype(object)


def mnist_small_plain(img, wts):
    """Exact integer logits of the small variant: convolution -> square ->
    dense 845 -> 10."""
    p = mnist_padded(img).astype(object)
    a1 = []
    for m in range(5):
        for y in range(MNIST_OUT):
            for x in range(MNIST_OUT):
                v = int((p[2 * y:2 * y + 5, 2 * x:2 * x + 5] * wts.conv_w[m].astype(object)).sum()) + int(wts.conv_b[m])
                a1.append(v * v)
    a1 = np.array(a1, dtype=object)
    return wts.w.astype(object).dot(a1) + wts.b.astype(object)


def head_plain(f, wts):
    """Exact integer logits of the 4096 -> 256 -> square -> 10 head."""
    h = wts.w1.astype(object).dot(np.asarray(f, dtype=object)) + wts.b1.astype(object)
    a = h * h
    return wts.w2.astype(object).dot(a) + wts.b2.astype(object)


# ----------------------------------------------------------------- schedule
@dataclasses.dataclass
class Schedule:
    N: int
    n_inputs: int
    ops: List[tuple]
    outputs: List[int]
    # where each result value ends up: list over outputs of {slot: label}
    out_slots: List[Dict[int, str]] = dataclasses.field(default_factory=list)

    def count(self, kind: str) -> int:
        """Ops of one kind; "rotate" counts hoisted rotations too."""
        if kind == "rotate":
            return sum(1 for op in self.ops if op[0] in ("rotate", "rotate_hoisted"))
        return sum(1 for op in self.ops if op[0] == kind)


class _Builder:
    def __init__(self, N, n_inputs, sums="sequential"):
        self.N = N
        self.n_inputs = n_inputs
        self.ops = []
        self.next = n_inputs
        # "sequential" or "hoisted": the form of rotate-and-sum and of the
        # combinations of shifted messages (`_rotate_and_sum`, `_combine_tree`)
        assert sums in ("sequential", "hoisted")
        self.sums = sums

    def reg(self):
        r = self.next
        self.next += 1
        return r

    def emit(self, *op):
        self.ops.append(tuple(op))
        return op[1]


def _rotate_and_sum(b: _Builder, src: int, steps: Sequence) -> int:
    """x += rot(x, k) for k in steps (left rotations / row swap).

    With b.sums == "hoisted" the same slots come from groups of up to three
    consecutive steps other than the row swap: after a group {s_1, .., s_k}
    the message is the sum over all subsets S of rot(x, sum(S)), formed as x
    plus its 2^k - 1 hoisted rotations by the non-empty subset sums (subsets in
    the order of their bit masks, bit i for s_i), added in that order; a row
    swap or a lone step stays x += rot(x, s)."""
    cur = src
    if b.sums == "sequential":
        for k in steps:
            r = b.emit("rotate", b.reg(), cur, k)
            cur = b.emit("add", b.reg(), cur, r)
        return cur
    i = 0
    while i < len(steps):
        grp = []
        while i < len(steps) and steps[i] != ROW_SWAP and len(grp) < 3:
            grp.append(steps[i])
            i += 1
        if len(grp) < 2:
            k = grp[0] if grp else steps[i]
            if not grp:
                i += 1
            r = b.emit("rotate", b.reg(), cur, k)
            cur = b.emit("add", b.reg(), cur, r)
            continue
        terms = [cur]
        for m in range(1, 1 << len(grp)):
            amount = sum(grp[j] for j in range(len(grp)) if m >> j & 1)
            terms.append(b.emit("rotate_hoisted", b.reg(), cur, amount))
        acc = terms[0]
        for t in terms[1:]:
            acc = b.emit("add", b.reg(), acc, t)
        cur = acc
    return cur


def _combine_tree(b: _Builder, regs: Sequence[int], unit: int) -> int:
    """sum_j rot(regs[j], -unit*j), built as a binary tree: at level l the odd
    member of each pair is rotated right by unit*2^l and added to the even one.
    Rotating right by unit*j is the composition of the rotations for the set
    bits of j, so the result is the same slot vector as the direct sum, with the
    same number of rotations (len-1) but only log2(len) distinct steps.
    With b.sums == "hoisted" (and more than two members): every member j >= 1
    rotated right by unit*j, then all added in order, one level."""
    if b.sums == "hoisted" and len(regs) > 2:
        acc = regs[0]
        rots = [b.emit("rotate", b.reg(), regs[j], -unit * j) for j in range(1, len(regs))]
        for r in rots:
            acc = b.emit("add", b.reg(), acc, r)
        return acc
    cur = list(regs)
    stride = unit
    while len(cur) > 1:
        nxt = []
        for i in range(0, len(cur), 2):
            if i + 1 < len(cur):
                r = b.emit("rotate", b.reg(), cur[i + 1], -stride)
                nxt.append(b.emit("add", b.reg(), cur[i], r))
            else:
                nxt.append(cur[i])
        cur = nxt
        stride *= 2
    return cur[0]


def _log2(x: int) -> int:
    assert x > 0 and x & (x - 1) == 0
    return x.bit_length() - 1


def _next_pow2(x: int) -> int:
    return 1 << max(0, (x - 1).bit_length())


def _stacked_rounds(b: _Builder, s: int, P: int, C: int, R: int, pos, w1, b1, recipe: str) -> int:
    """Dense layer on C stacked copies of its input (block c = slots P c ..
    P c + P - 1, input i at offset pos[i]) in R rounds of stacked vector - row
    major (Sec. 4.2.2): round rho multiplies by the rows C rho + c laid out in
    block c.  Returns the combined message, value C rho + c at slot P c + rho.

    recipe "full": each round is summed over its whole block (rotations 1 ..
    P/2), masked to slot P c with the bias added there, and the rounds are
    combined by shifting round rho right by rho.
    recipe "shared": each round is summed only within groups of G =
    next_pow2(R) slots (rotations 1 .. G/2), masked to the group starts
    P c + G m (bias at P c), the rounds are shifted right by rho into the free
    offsets of those groups, and one rotate-and-sum over G .. P/2 finishes
    every round's block sum at once: slot P c + rho then holds
    sum_m sum_{d<G} round_rho[P c + G m + d], the full block sum.  Slots other
    than P c + rho hold partial sums (garbage)."""
    out_dim = w1.shape[0]
    G = _next_pow2(R) if recipe == "shared" else P
    rounds = []
    for rho in range(R):
        rows, mask, bias = {}, {}, {}
        for c in range(C):
            j = C * rho + c
            if j >= out_dim:
                continue
            for i, p_i in enumerate(pos):
                rows[P * c + p_i] = int(w1[j, i])
            for m in range(P // G):
                mask[P * c + G * m] = 1
            bias[P * c] = int(b1[j])
        z = b.emit("mul_plain", b.reg(), s, rows)
        z = _rotate_and_sum(b, z, [1 << k for k in range(_log2(G))])
        z = b.emit("mul_plain", b.reg(), z, mask)
        z = b.emit("add_plain", b.reg(), z, bias)
        rounds.append(z)
    h = _combine_tree(b, rounds, 1)
    if recipe == "shared":
        h = _rotate_and_sum(b, h, [1 << k for k in range(_log2(G), _log2(P))])
    return h


def _interleaved_output(b: _Builder, h: int, N: int, P: int, C: int, R: int, w2, b2, recipe: str):
    """Last dense layer on an interleaved vector (value C rho + c at slot
    P c + rho), Interleaved vector - Row Major (Sec. 4.2.2).  Returns
    (outputs, out_slots).

    recipe "full": per output o, the product with the row permuted to the
    interleaved layout and a rotate-and-sum over 1 .. G/2 (G = next_pow2(R)),
    P .. and the row swap when the blocks fill both rows -> logit o at slot 0
    of message o.
    recipe "shared": one packed message.  Copy o of the input is the input
    rotated right by G o, all copies hoisted rotations of the one input
    (bfv.rotate_hoisted: they share its decomposition), multiplied by row o
    laid out at slots P c + G o + rho; the products are added and one
    rotate-and-sum over the same steps leaves logit o at slot G o."""
    n_out, in_dim = w2.shape
    G = _next_pow2(R)
    coll = [1 << k for k in range(_log2(G))]
    coll += [P << k for k in range(_log2(N // 2) - _log2(P)) if (P << k) < P * C]
    if P * C > N // 2:
        coll.append(ROW_SWAP)
    if recipe == "full":
        outs = []
        for o in range(n_out):
            rows = {P * c + rho: int(w2[o, C * rho + c])
                    for rho in range(R) for c in range(C) if C * rho + c < in_dim}
            z = b.emit("mul_plain", b.reg(), h, rows)
            z = _rotate_and_sum(b, z, coll)
            z = b.emit("add_plain", b.reg(), z, {0: int(b2[o])})
            outs.append(z)
        return outs, [{0: f"logit{o}"} for o in range(n_out)]
    assert G * n_out <= P
    copies = [h] + [b.emit("rotate_hoisted", b.reg(), h, -G * o) for o in range(1, n_out)]
    acc = None
    for o in range(n_out):
        rows = {P * c + G * o + rho: int(w2[o, C * rho + c])
                for rho in range(R) for c in range(C) if C * rho + c < in_dim}
        z = b.emit("mul_plain", b.reg(), copies[o], rows)
        acc = z if acc is None else b.emit("add", b.reg(), acc, z)
    z = _rotate_and_sum(b, acc, coll)
    z = b.emit("add_plain", b.reg(), z, {G * o: int(b2[o]) for o in range(n_out)})
    return [z], [{G * o: f"logit{o}" for o in range(n_out)}]


def dense64_inputs(x, N):
    """Client side: the 64-vector stacked N/64 times (stacked representation,
    Sec. 4.2.1, with d = 6): slot i holds x[i mod 64]."""
    x = np.asarray(x, dtype=np.int64)
    return [{s: int(x[s % 64]) for s in range(N)}]


def dense64_schedule(W, N: int = 4096, sums: str = "sequential") -> Schedule:
    """Stacked vector - row major (Sec. 4.2.2): one point-wise product with the
    64 rows of W laid out row j at slots 64j..64j+63, then rotations of size
    1, 2, ..., 32 and additions; value j ends at slot 64j (interleaved), then
    squared."""
    assert N == 4096
    b = _Builder(N, 1, sums)
    W = np.asarray(W, dtype=np.int64)
    rows = {64 * j + i: int(W[j, i]) for j in range(64) for i in range(64)}
    z = b.emit("mul_plain", b.reg(), 0, rows)
    z = _rotate_and_sum(b, z, [1, 2, 4, 8, 16, 32])
    y = b.emit("square", b.reg(), z)
    return Schedule(N, 1, b.ops, [y], [{64 * j: f"y{j}" for j in range(64)}])


# MNIST (N = 16384): slots are a 2 x 8192 matrix; slot index r*8192 + i.
def conv_representation(img, k: int, stride: int):
    """Convolution representation (Sec. 4.2.1) of a 2-D input for a k x k
    window at the given stride: k*k messages; message a*k+b holds, at entry
    y*n_out + x, the input value [stride*y + a][stride*x + b], so that
    sum_{a,b} w[a,b] * message(a,b) is the convolution output at (y, x).
    Returns a list of 1-D integer arrays."""
    img = np.asarray(img)
    n_out = (img.shape[0] - k) // stride + 1
    msgs = []
    for a in range(k):
        for b in range(k):
            msgs.append(np.array([img[stride * y + a, stride * x + b]
                                  for y in range(n_out) for x in range(n_out)]))
    return msgs


def mnist_inputs(img, N=16384):
    """Client side convolution representation of the zero-padded image for the
    5x5, stride-2 window: message 5a+b holds at slot 13y+x the padded pixel
    [2y+a][2x+b]."""
    return [{i: int(v) for i, v in enumerate(m)}
            for m in conv_representation(mnist_padded(img), 5, 2)]


def mnist_schedule(wts, N: int = 16384, recipe: str = "full", sums: str = "sequential") -> Schedule:
    """The LoLa MNIST pipeline of Table 1, laid out for N = 16384 as the paper
    does for LoLa-Dense in App. C (16 stacked copies, 7 rounds):
      conv:    per map, sum_{a,b} w[m,a,b] * M_{a,b} (message x scalar) + bias
      combine: map m rotated right by 169 m and added (4 rotations, as a
               binary tree over steps 169, 338, 676)
      square
      stack:   copies at stride 1024 by rotating right 1024, 2048, 4096 and a
               row swap (16 copies)
      dense1:  7 rounds of stacked vector - row major with rows 16 rho + c in
               block c, combined into an interleaved vector, value 16 rho + c
               at slot 1024 c + rho (`_stacked_rounds`)
      square
      dense2:  interleaved vector - row major (`_interleaved_output`).
    recipe "full" is the layout the paper describes: every round summed over
    its block (10 rotations), masked, combined (6 rotations), and one message
    per logit (7 rotations each) -> 154 rotations.  recipe "shared" sums the
    rounds only within groups of 8 slots before combining them and finishes
    with one shared rotate-and-sum, and packs the ten logits into one message
    -> 58 rotations, the same values at the valid slots.
    sums "hoisted": every rotate-and-sum and combination in the hoisted form
    (`_rotate_and_sum`, `_combine_tree`)."""
    assert N == 16384
    b = _Builder(N, 25, sums)
    maps = []
    for m in range(5):
        acc = None
        for a in range(5):
            for c in range(5):
                t = b.emit("mul_scalar", b.reg(), 5 * a + c, int(wts.conv_w[m, a, c]))
                acc = t if acc is None else b.emit("add", b.reg(), acc, t)
        acc = b.emit("add_plain", b.reg(), acc, {s: int(wts.conv_b[m]) for s in range(169)})
        maps.append(acc)
    y = _combine_tree(b, maps, 169)
    y = b.emit("square", b.reg(), y)
    s = _rotate_and_sum(b, y, [-1024, -2048, -4096, ROW_SWAP])
    h = _stacked_rounds(b, s, 1024, 16, 7, range(845), wts.w1, wts.b1, recipe)
    h = b.emit("square", b.reg(), h)
    outs, slots = _interleaved_output(b, h, N, 1024, 16, 7, wts.w2, wts.b2, recipe)
    return Schedule(N, 25, b.ops, outs, slots)


def mnist_small_schedule(wts, N: int = 16384, sums: str = "sequential") -> Schedule:
    """LoLa-Small (Sec. 4.3: a convolution layer, the square activation and one
    dense layer), laid out like the first half of `mnist_schedule`:
      conv, combine (tree over 169, 338, 676), square, stack 16 copies at
      stride 1024;
      dense:   one round of stacked vector - row major: the product with row o
               in block o (o < 10), rotate-and-sum 1..512, bias added at slot
               1024 o -> logit o at slot 1024 o of the one output message."""
    assert N == 16384
    b = _Builder(N, 25, sums)
    maps = []
    for m in range(5):
        acc = None
        for a in range(5):
            for c in range(5):
                t = b.emit("mul_scalar", b.reg(), 5 * a + c, int(wts.conv_w[m, a, c]))
                acc = t if acc is None else b.emit("add", b.reg(), acc, t)
        acc = b.emit("add_plain", b.reg(), acc, {s: int(wts.conv_b[m]) for s in range(169)})
        maps.append(acc)
    y = _combine_tree(b, maps, 169)
    y = b.emit("square", b.reg(), y)
    s = _rotate_and_sum(b, y, [-1024, -2048, -4096, ROW_SWAP])
    rows = {1024 * o + i: int(wts.w[o, i]) for o in range(10) for i in range(845)}
    z = b.emit("mul_plain", b.reg(), s, rows)
    z = _rotate_and_sum(b, z, [1 << k for k in range(10)])
    z = b.emit("add_plain", b.reg(), z, {1024 * o: int(wts.b[o]) for o in range(10)})
    return Schedule(N, 25, b.ops, [z], [{1024 * o: f"logit{o}" for o in range(10)}])


# LoLa-Dense (App. C): the image arrives as one dense message and the
# convolution representation is built from it with masks and rotations.
MNIST_DENSE_OFFSETS = (0, 1, 29, 30, 754)   # placement of map m after the convolution
MNIST_DENSE_BLOCK = 2048                    # stacking period: 754 + 720 < 2048


def mnist_dense_inputs(img, N=16384):
    """Dense representation: the zero-padded 29 x 29 image row by row, padded
    pixel (i, j) at slot 29 i + j."""
    p = mnist_padded(img)
    return [{29 * i + j: int(p[i, j]) for i in range(29) for j in range(29) if p[i, j]}]


def mnist_dense_schedule(wts, N: int = 16384, recipe: str = "full", sums: str = "sequential") -> Schedule:
    """LoLa-Dense (App. C, Table 3) for N = 16384:
      masks:   message (a, b) = the input rotated left by 29 a + b (so padded
               pixel (2y + a, 2x + b) sits at slot 58 y + 2 x) times the 0/1
               mask of the window corners {58 y + 2 x : y, x < 13}; 24
               rotations of the one input, hoisted (they share its
               decomposition), and 25 products;
      conv:    per map, sum_{a,b} w[m,a,b] * message(a,b) + bias at the corners;
      combine: map m rotated right by (0, 1, 29, 30, 754)[m] and added, so the
               845 values occupy distinct slots below 2048 (4 rotations);
      square;
      stack:   8 copies at stride 2048 (rotations right 2048, 4096, row swap);
      dense1:  13 rounds of stacked vector - row major: block c holds row
               8 rho + c laid out on the combined positions, combined into
               value 8 rho + c at slot 2048 c + rho (`_stacked_rounds`);
      square;
      dense2:  interleaved vector - row major (`_interleaved_output`).
    recipe "full": 256 rotations (each round summed over 1 .. 1024, one
    message per logit); recipe "shared": 118 rotations."""
    assert N == 16384
    P, C = MNIST_DENSE_BLOCK, N // MNIST_DENSE_BLOCK
    R = (100 + C - 1) // C
    b = _Builder(N, 1, sums)
    corners = {58 * y + 2 * x: 1 for y in range(MNIST_OUT) for x in range(MNIST_OUT)}
    msgs = []
    for a in range(5):
        for c in range(5):
            r = 29 * a + c
            src = 0 if r == 0 else b.emit("rotate_hoisted", b.reg(), 0, r)
            msgs.append(b.emit("mul_plain", b.reg(), src, corners))
    maps = []
    for m in range(5):
        acc = None
        for k in range(25):
            t = b.emit("mul_scalar", b.reg(), msgs[k], int(wts.conv_w[m, k // 5, k % 5]))
            acc = t if acc is None else b.emit("add", b.reg(), acc, t)
        acc = b.emit("add_plain", b.reg(), acc, {s: int(wts.conv_b[m]) for s in corners})
        maps.append(acc)
    y = maps[0]
    for m in range(1, 5):
        r = b.emit("rotate", b.reg(), maps[m], -MNIST_DENSE_OFFSETS[m])
        y = b.emit("add", b.reg(), y, r)
    y = b.emit("square", b.reg(), y)
    s = _rotate_and_sum(b, y, [-2048, -4096, ROW_SWAP])
    pos = [MNIST_DENSE_OFFSETS[m] + 58 * yy + 2 * xx
           for m in range(5) for yy in range(MNIST_OUT) for xx in range(MNIST_OUT)]
    h = _stacked_rounds(b, s, P, C, R, pos, wts.w1, wts.b1, recipe)
    h = b.emit("square", b.reg(), h)
    outs, slots = _interleaved_output(b, h, N, P, C, R, wts.w2, wts.b2, recipe)
    return Schedule(N, 1, b.ops, outs, slots)


# CIFAR-shaped network (Sec. 4.4, App. D, collapsed form): 8x8x3 convolution
# at stride 2 -> square -> 6xkx convolution at stride 2 over all maps -> square
# -> dense -> 10.  The 32x32 image is zero-padded by one pixel on every side
# (34x34), so the first convolution has 14x14 outputs (83 maps: 16268 values)
# and the second 5x5 (163 maps: 4075 values).
CIFAR_PAD = 34


def cifar_padded(img):
    img = np.asarray(img, dtype=np.int64)
    c, h, w = img.shape
    p = np.zeros((c, h + 2, w + 2), dtype=np.int64)
    p[:, 1:h + 1, 1:w + 1] = img
    return p


def _conv_plain(x, w, b, stride):
    """x: [C][H][H] integers (object), w: [M][C][k][k] -> [M][n][n]."""
    C, H, _ = x.shape
    M, _, k, _ = w.shape
    n = (H - k) // stride + 1
    out = np.zeros((M, n, n), dtype=object)
    wo = w.astype(object)
    for m in range(M):
        for y in range(n):
            for xx in range(n):
                out[m, y, xx] = int((x[:, stride * y:stride * y + k, stride * xx:stride * xx + k] * wo[m]).sum()) + int(b[m])
    return out


def cifar_plain(padded, wts):
    """Exact integer logits of the CIFAR-shaped network on an already padded
    [3][H][H] input."""
    a1 = _conv_plain(np.asarray(padded).astype(object), wts.conv1_w, wts.conv1_b, 2)
    a1 = a1 * a1
    a2 = _conv_plain(a1, wts.conv2_w, wts.conv2_b, 2)
    a2 = (a2 * a2).reshape(-1)          # index 25 m + 5 y + x at full size
    return wts.w3.astype(object).dot(a2) + wts.b3.astype(object)


def cifar_inputs(padded):
    """Convolution representation of the padded input for the 8x8 window at
    stride 2: message 64 c + 8 a + b holds padded[c][2y+a][2x+b] at slot
    n1*y + x."""
    p = np.asarray(padded)
    return [{i: int(v) for i, v in enumerate(m)}
            for c in range(p.shape[0]) for m in conv_representation(p[c], 8, 2)]


def cifar_layout(m1, n1, N):
    """Where the first convolution's maps go after combining: map m in message
    m // (2 R), row (m mod 2R) // R, block (m mod R) of n1*n1 slots, with R
    maps per slot row (rotations stay inside a row)."""
    V1 = n1 * n1
    R = (N // 2) // V1
    return [(m // (2 * R), (m % (2 * R)) // R * (N // 2) + (m % R) * V1) for m in range(m1)], R


def cifar_schedule(wts, n_in: int, N: int = 16384) -> Schedule:
    """LoLa on the CIFAR-shaped network (Sec. 4.4), for a padded input of
    n_in x n_in pixels per channel:
      conv1:   per map, sum over the 3*64 convolution messages (message x
               scalar) + bias at slots 0..n1^2-1;
      combine: within a slot row, maps as blocks of n1^2 slots (binary tree of
               right rotations); the second row's maps brought over by the row
               swap; 2R maps per message (R per row);
      square   (one product per message);
      conv2:   dense vector - row major: per output (map, y, x), the products
               of every message with its weights at the window's slots, summed,
               then rotate-and-sum over 1 .. N/4 and the row swap, so every
               slot holds the output;
      gather:  output j multiplied by the one-hot plaintext of slot j, all
               summed into one dense message, then the biases added at once
               (one plaintext: adding them one output at a time would give
               the same slots but other ciphertext words, since the scaled
               plaintext floor(Q/t) m depends on m's representative in [0, t));
      square;
      dense:   per logit, the product with its row, rotate-and-sum over the
               next power of two above the hidden size -> logit at slot 0."""
    b = _Builder(N, wts.conv1_w.shape[1] * wts.conv1_w.shape[2] ** 2)
    gathered, H = _cifar_front(b, wts, n_in, N)
    h = b.emit("square", b.reg(), gathered)
    steps = [1 << i for i in range(max(1, int(np.ceil(np.log2(H)))))]
    outs = []
    for o in range(wts.w3.shape[0]):
        z = b.emit("mul_plain", b.reg(), h, {j: int(wts.w3[o, j]) for j in range(H)})
        z = _rotate_and_sum(b, z, steps)
        z = b.emit("add_plain", b.reg(), z, {0: int(wts.b3[o])})
        outs.append(z)
    return Schedule(N, b.n_inputs, b.ops, outs, [{0: f"logit{o}"} for o in range(len(outs))])


def _cifar_front(b: _Builder, wts, n_in: int, N: int):
    """The CIFAR-shaped network up to the second convolution's outputs with
    their biases (before its square): one dense message, output j at slot
    j.  Returns (register, number of outputs)."""
    m1, C, k1, _ = wts.conv1_w.shape
    m2, _, k2, _ = wts.conv2_w.shape
    n1 = (n_in - k1) // 2 + 1
    n2 = (n1 - k2) // 2 + 1
    V1, V2 = n1 * n1, n2 * n2
    H = m2 * V2
    place, R = cifar_layout(m1, n1, N)
    G = max(g for g, _ in place) + 1
    maps = []
    for m in range(m1):
        acc = None
        for c in range(C):
            for a in range(k1):
                for cc in range(k1):
                    t = b.emit("mul_scalar", b.reg(), c * k1 * k1 + a * k1 + cc, int(wts.conv1_w[m, c, a, cc]))
                    acc = t if acc is None else b.emit("add", b.reg(), acc, t)
        maps.append(b.emit("add_plain", b.reg(), acc, {s: int(wts.conv1_b[m]) for s in range(V1)}))
    msgs = []
    for g in range(G):
        rows = []
        for r in range(2):
            ms = [maps[m] for m in range(m1) if place[m][0] == g and place[m][1] // (N // 2) == r]
            if ms:
                rows.append(_combine_tree(b, ms, V1))
        y = rows[0]
        if len(rows) == 2:
            sw = b.emit("rotate", b.reg(), rows[1], ROW_SWAP)
            y = b.emit("add", b.reg(), y, sw)
        msgs.append(b.emit("square", b.reg(), y))
    full = [1 << i for i in range(int(np.log2(N // 2)))] + [ROW_SWAP]
    gathered = None
    for j in range(H):
        mo, yx = divmod(j, V2)
        y2, x2 = divmod(yx, n2)
        z = None
        for g in range(G):
            row = {}
            for m in range(m1):
                if place[m][0] != g:
                    continue
                base = place[m][1]
                for a in range(k2):
                    for cc in range(k2):
                        row[base + n1 * (2 * y2 + a) + 2 * x2 + cc] = int(wts.conv2_w[mo, m, a, cc])
            t = b.emit("mul_plain", b.reg(), msgs[g], row)
            z = t if z is None else b.emit("add", b.reg(), z, t)
        z = _rotate_and_sum(b, z, full)
        z = b.emit("mul_plain", b.reg(), z, {j: 1})
        gathered = z if gathered is None else b.emit("add", b.reg(), gathered, z)
    gathered = b.emit("add_plain", b.reg(), gathered, {j: int(wts.conv2_b[j // V2]) for j in range(H)})
    return gathered, H


# Chains of dense layers and squares on one query, with the two recipes that
# take a vector in one representation and give it in the other (Sec. 4.2.2):
# dense vector - row major turns a dense input into a sparse output, sparse
# vector - column major turns a sparse input into a dense output.
def dense_chain_plain(x, layers):
    """The plaintext network on integers: layers are ("dense", W, b) (b may be
    None) and ("square",)."""
    a = np.asarray(x, dtype=np.int64).astype(object)
    for ly in layers:
        if ly[0] == "square":
            a = a * a
        else:
            W = np.asarray(ly[1], dtype=np.int64).astype(object)
            a = W.dot(a)
            if ly[2] is not None:
                a = a + np.asarray(ly[2], dtype=np.int64).astype(object)
    return a


def _dense_row_major_full(b: _Builder, src: int, W, bias, N: int, pos=None) -> List[int]:
    """Dense vector - row major (Sec. 4.2.2) with the output in sparse form:
    per row j, the product with row j (value W[j, i] at the input's slot
    pos[i], slot i by default), then a rotate-and-sum over 1, 2, ..., N/4
    and the row swap, after which every slot holds the dot product; the bias
    is added in every slot.  One message per row."""
    full = [1 << i for i in range(_log2(N // 2))] + [ROW_SWAP]
    pos = list(range(W.shape[1])) if pos is None else list(pos)
    outs = []
    for j in range(W.shape[0]):
        z = b.emit("mul_plain", b.reg(), src, {pos[i]: int(W[j, i]) for i in range(W.shape[1])})
        z = _rotate_and_sum(b, z, full)
        if bias is not None:
            z = b.emit("add_plain", b.reg(), z, {s: int(bias[j]) for s in range(N)})
        outs.append(z)
    return outs


def _sparse_column_major(b: _Builder, srcs: Sequence[int], W, bias) -> int:
    """Sparse vector - column major (Sec. 4.2.2): value i of the input is the
    message srcs[i] with v_i in every slot, so W v = sum_i v_i c^i is one
    product of message i with column i (value W[j, i] at slot j) per input
    and the sum of the products; the bias is added at slots 0..r-1.  The
    result is dense: value j at slot j, zero elsewhere."""
    acc = None
    for i, s in enumerate(srcs):
        t = b.emit("mul_plain", b.reg(), s, {j: int(W[j, i]) for j in range(W.shape[0])})
        acc = t if acc is None else b.emit("add", b.reg(), acc, t)
    if bias is not None:
        acc = b.emit("add_plain", b.reg(), acc, {j: int(bias[j]) for j in range(W.shape[0])})
    return acc


def dense_chain_inputs(x, N: int, sparse_input: bool):
    """Client side: the dense representation (value i at slot i, one message)
    or the sparse one (message i with x_i in every slot)."""
    x = np.asarray(x, dtype=np.int64)
    if sparse_input:
        return [{s: int(v) for s in range(N)} for v in x]
    return [{i: int(v) for i, v in enumerate(x)}]


def dense_chain_schedule(layers, N: int, sparse_input: bool) -> Schedule:
    """Each dense layer takes the recipe its input's representation calls
    for: sparse vector - column major on a sparse input (k products, no
    rotation, dense result), dense vector - row major on a dense input (a
    full rotate-and-sum per row, sparse result); a square acts on every
    message of the representation.  The outputs are the r messages of a
    sparse result (value j in every slot of message j) or the one message of
    a dense result (value j at slot j)."""
    k = np.asarray(layers[0][1]).shape[1]
    b = _Builder(N, k if sparse_input else 1)
    regs, sparse = (list(range(k)), True) if sparse_input else ([0], False)
    for ly in layers:
        if ly[0] == "square":
            regs = [b.emit("square", b.reg(), r) for r in regs]
            continue
        W = np.asarray(ly[1], dtype=np.int64)
        if sparse:
            regs, sparse = [_sparse_column_major(b, regs, W, ly[2])], False
        else:
            regs, sparse = _dense_row_major_full(b, regs[0], W, ly[2], N), True
    r = len(regs) if sparse else np.asarray([ly for ly in layers if ly[0] == "dense"][-1][1]).shape[0]
    out_slots = [{0: f"y{j}"} for j in range(r)] if sparse else [{j: f"y{j}" for j in range(r)}]
    return Schedule(N, b.n_inputs, b.ops, regs, out_slots)


# The MNIST-shaped convolution front end followed by any chain of dense layers
# and squares (the first layer after the convolution's square is dense).
def conv_chain_plain(img, conv_w, conv_b, layers):
    """Exact integers: the 5x5 stride-2 convolution with five maps over the
    zero-padded 29x29 image, squared, flattened (index 169 m + 13 y + x),
    then the chain (`dense_chain_plain`)."""
    p = mnist_padded(img).astype(object)
    conv = np.zeros((5, MNIST_OUT, MNIST_OUT), dtype=object)
    for m in range(5):
        for y in range(MNIST_OUT):
            for x in range(MNIST_OUT):
                win = p[2 * y:2 * y + 5, 2 * x:2 * x + 5]
                conv[m, y, x] = int((win * np.asarray(conv_w[m]).astype(object)).sum()) + int(conv_b[m])
    return dense_chain_plain((conv * conv).reshape(845), layers)


def conv_chain_schedule(conv_w, conv_b, layers, N: int = 16384, recipe: str = "full") -> Schedule:
    """The front end of `mnist_schedule` (convolution, combine, square, 16
    stacked copies at stride 1024) and the first dense layer as its stacked
    rounds (`_stacked_rounds`, recipe "full" or "shared"), giving the
    interleaved hidden vector, value 16 rho + c at slot 1024 c + rho; every
    later dense layer takes the recipe its input's representation calls for
    (Sec. 4.2.2): dense vector - row major on the interleaved or dense vector
    (`_dense_row_major_full` with the values' slots, a sparse result), sparse
    vector - column major on a sparse one (a dense result, value j at slot
    j); a square squares every message."""
    assert N == 16384 and layers[0][0] == "dense"
    b = _Builder(N, 25)
    maps = []
    for m in range(5):
        acc = None
        for a in range(5):
            for c in range(5):
                t = b.emit("mul_scalar", b.reg(), 5 * a + c, int(conv_w[m][a][c]))
                acc = t if acc is None else b.emit("add", b.reg(), acc, t)
        acc = b.emit("add_plain", b.reg(), acc, {s: int(conv_b[m]) for s in range(169)})
        maps.append(acc)
    y = _combine_tree(b, maps, 169)
    y = b.emit("square", b.reg(), y)
    s = _rotate_and_sum(b, y, [-1024, -2048, -4096, ROW_SWAP])
    W1 = np.asarray(layers[0][1], dtype=np.int64)
    R = -(-W1.shape[0] // 16)
    h = _stacked_rounds(b, s, 1024, 16, R, range(845), W1, layers[0][2], recipe)
    return _chain_tail(b, h, [1024 * (j % 16) + j // 16 for j in range(W1.shape[0])], layers[1:])


def _chain_tail(b: _Builder, src: int, pos, layers) -> Schedule:
    """The rest of a network from one dense message (value j at slot pos[j]):
    each dense layer with the recipe its input's representation calls for
    (Sec. 4.2.2), dense vector - row major on a dense vector (a sparse
    result: one message per value, the value in every slot), sparse vector -
    column major on a sparse one (a dense result, value j at slot j); a
    square squares every message."""
    regs, sparse, pos, width = [src], False, list(pos), len(pos)
    for ly in layers:
        if ly[0] == "square":
            regs = [b.emit("square", b.reg(), r) for r in regs]
            continue
        W = np.asarray(ly[1], dtype=np.int64)
        if sparse:
            regs, sparse, pos = [_sparse_column_major(b, regs, W, ly[2])], False, list(range(W.shape[0]))
        else:
            regs, sparse = _dense_row_major_full(b, regs[0], W, ly[2], b.N, pos), True
        width = W.shape[0]
    out_slots = [{0: f"y{j}"} for j in range(width)] if sparse else [{pos[j]: f"y{j}" for j in range(width)}]
    return Schedule(b.N, b.n_inputs, b.ops, regs, out_slots)


def cifar_chain_plain(padded, wts, tail):
    """Exact integers: the CIFAR-shaped network's two convolutions (the
    first squared), the second's outputs flattened (index V2 m + n2 y + x),
    then the chain `tail` of dense layers and squares (`dense_chain_plain`)."""
    a1 = _conv_plain(np.asarray(padded).astype(object), wts.conv1_w, wts.conv1_b, 2)
    a2 = _conv_plain(a1 * a1, wts.conv2_w, wts.conv2_b, 2)
    return dense_chain_plain(a2.reshape(-1), tail)


def cifar_chain_schedule(wts, tail, n_in: int, N: int = 16384) -> Schedule:
    """The CIFAR-shaped front end of `cifar_schedule` up to the second
    convolution's dense output (before its square), then the chain `tail`
    (`_chain_tail`), e.g. SQUARE, DENSE, SQUARE, DENSE."""
    b = _Builder(N, wts.conv1_w.shape[1] * wts.conv1_w.shape[2] ** 2)
    gathered, H = _cifar_front(b, wts, n_in, N)
    return _chain_tail(b, gathered, range(H), tail)


# Transfer-learning head (N = 16384, 4 queries per ciphertext, query q in the
# 4096-slot block starting at slot 4096 q).
HEAD_BLOCK = 4096


def head_inputs(features, N=16384):
    """Dense representation, one block per query (up to 4 per message)."""
    f = np.asarray(features, dtype=np.int64)
    assert f.shape[0] <= N // HEAD_BLOCK
    return [{HEAD_BLOCK * q + i: int(f[q, i]) for q in range(f.shape[0]) for i in range(HEAD_BLOCK)}]


def head_schedule(wts, N: int = 16384, n_hidden: int | None = None, n_out: int = 10,
                  sums: str = "sequential") -> Schedule:
    """Dense vector - row major (Sec. 4.2.2) for 4096 -> 256: per hidden unit
    j, product with row j repeated in every block, rotate-and-sum over
    1..2048 (each block's sum lands at its first slot), mask, then rotate
    right by j and add, as a binary tree (interleaved result, h_j of query q at slot 4096 q + j),
    bias, square; then interleaved vector - row major for 256 -> 10 with
    rotate-and-sum over 1..128 (logit o of query q at slot 4096 q).
    n_hidden < 256 builds a truncated head (for quick checks)."""
    assert N == 16384
    nb = N // HEAD_BLOCK
    nh = wts.w1.shape[0] if n_hidden is None else n_hidden
    b = _Builder(N, 1, sums)
    hidden = []
    for j in range(nh):
        rows = {HEAD_BLOCK * q + i: int(wts.w1[j, i]) for q in range(nb) for i in range(HEAD_BLOCK)}
        z = b.emit("mul_plain", b.reg(), 0, rows)
        z = _rotate_and_sum(b, z, [1 << k for k in range(12)])
        z = b.emit("mul_plain", b.reg(), z, {HEAD_BLOCK * q: 1 for q in range(nb)})
        hidden.append(z)
    acc = _combine_tree(b, hidden, 1)
    acc = b.emit("add_plain", b.reg(), acc,
                 {HEAD_BLOCK * q + j: int(wts.b1[j]) for q in range(nb) for j in range(nh)})
    h = b.emit("square", b.reg(), acc)
    steps = [1 << k for k in range(int(np.ceil(np.log2(max(nh, 2)))))]
    outs = []
    for o in range(n_out):
        rows = {HEAD_BLOCK * q + j: int(wts.w2[o, j]) for q in range(nb) for j in range(nh)}
        z = b.emit("mul_plain", b.reg(), h, rows)
        z = _rotate_and_sum(b, z, steps)
        z = b.emit("add_plain", b.reg(), z, {HEAD_BLOCK * q: int(wts.b2[o]) for q in range(nb)})
        outs.append(z)
    return Schedule(N, 1, b.ops, outs,
                    [{HEAD_BLOCK * q: f"q{q}_logit{o}" for q in range(nb)} for o in range(n_out)])


def head_stacked_inputs(features, N=16384):
    """Stacked representation of one query (Sec. 4.2.1): the feature vector
    repeated in every block of HEAD_BLOCK slots (the client sends the copies)."""
    f = np.asarray(features, dtype=np.int64).reshape(-1)
    return [{HEAD_BLOCK * c + i: int(f[i]) for c in range(N // HEAD_BLOCK) for i in range(f.size)}]


def head_stacked_schedule(wts, N: int = 16384, n_hidden: int | None = None, n_out: int = 10,
                          sums: str = "sequential") -> Schedule:
    """The same head, one query per message, with the stacked vector - row
    major method (Sec. 4.2.2) for the hidden layer:
      rounds:  C = N / 4096 copies; round rho multiplies by rows C rho + c in
               block c, rotate-and-sum over 1..2048, keeps slot 4096 c (mask),
               adds the bias there;
      combine: round rho rotated right by rho (binary tree) -> hidden unit
               C rho + c at slot 4096 c + rho;
      square;
      output:  interleaved vector - row major: per logit, the product with
               the row in that layout and rotate-and-sum over 1 .. (rounds)/2,
               the block strides and the row swap -> logit at slot 0."""
    assert N == 16384
    P = HEAD_BLOCK
    C = N // P
    nh = wts.w1.shape[0] if n_hidden is None else n_hidden
    R = (nh + C - 1) // C
    b = _Builder(N, 1, sums)
    rounds = []
    for rho in range(R):
        rows, mask, bias = {}, {}, {}
        for c in range(C):
            j = C * rho + c
            if j >= nh:
                continue
            for i in range(wts.w1.shape[1]):
                rows[P * c + i] = int(wts.w1[j, i])
            mask[P * c] = 1
            bias[P * c] = int(wts.b1[j])
        z = b.emit("mul_plain", b.reg(), 0, rows)
        z = _rotate_and_sum(b, z, [1 << k for k in range(12)])
        z = b.emit("mul_plain", b.reg(), z, mask)
        z = b.emit("add_plain", b.reg(), z, bias)
        rounds.append(z)
    h = _combine_tree(b, rounds, 1)
    h = b.emit("square", b.reg(), h)
    coll = [1 << k for k in range(int(np.ceil(np.log2(max(R, 2)))))]
    coll += [s for s in (P, 2 * P, 4 * P) if s < N // 2 and s < P * C]
    if P * C > N // 2:
        coll.append(ROW_SWAP)
    outs = []
    for o in range(n_out):
        rows = {}
        for rho in range(R):
            for c in range(C):
                j = C * rho + c
                if j < nh:
                    rows[P * c + rho] = int(wts.w2[o, j])
        z = b.emit("mul_plain", b.reg(), h, rows)
        z = _rotate_and_sum(b, z, coll)
        z = b.emit("add_plain", b.reg(), z, {0: int(wts.b2[o])})
        outs.append(z)
    return Schedule(N, 1, b.ops, outs, [{0: f"logit{o}"} for o in range(n_out)])


# ------------------------------------------------------------- interpreters
def dense_slots(sparse: Dict[int, int], N: int, t: int) -> np.ndarray:
    v = np.zeros(N, dtype=np.int64)
    for k, x in sparse.items():
        v[k] = int(x) % t
    return v


def rotate_slots(v: np.ndarray, step) -> np.ndarray:
    """Slot-level rotation: left by step within each row; row swap."""
    n2 = len(v) // 2
    if step == ROW_SWAP:
        return np.concatenate([v[n2:], v[:n2]])
    k = int(step) % n2
    return np.concatenate([np.roll(v[:n2], -k), np.roll(v[n2:], -k)])


def run_slots(sched: Schedule, inputs: Sequence[Dict[int, int]], t: int):
    """Every register's full slot vector mod t; returns (outputs, registers)."""
    N = sched.N
    reg = {i: dense_slots(inputs[i], N, t) for i in range(sched.n_inputs)}
    for op in sched.ops:
        k = op[0]
        if k == "mul_scalar":
            reg[op[1]] = (reg[op[2]] * (int(op[3]) % t)) % t
        elif k == "add":
            reg[op[1]] = (reg[op[2]] + reg[op[3]]) % t
        elif k == "add_plain":
            reg[op[1]] = (reg[op[2]] + dense_slots(op[3], N, t)) % t
        elif k == "mul_plain":
            reg[op[1]] = (reg[op[2]] * dense_slots(op[3], N, t)) % t
        elif k in ("rotate", "rotate_hoisted"):
            reg[op[1]] = rotate_slots(reg[op[2]], op[3])
        elif k == "square":
            reg[op[1]] = (reg[op[2]] * reg[op[2]]) % t
        else:
            raise ValueError(k)
    return [reg[o] for o in sched.outputs], reg


def galois_elements(sched: Schedule) -> List[int]:
    gs = sorted({bfv.galois_element(sched.N, op[3]) for op in sched.ops if op[0] in ("rotate", "rotate_hoisted")})
    return [g for g in gs if g != 1]


def _sources(op):
    return [op[2], op[3]] if op[0] == "add" else [op[2]]


def run_ciphertexts(ctx: bfv.Context, keys: bfv.Keys, sched: Schedule, cts, keep=False, progress=None):
    """Evaluates the schedule on ciphertexts with the oracle's operations.
    Intermediate registers are dropped after their last use unless keep;
    progress(done, total) is called every 250 ops when given."""
    last_use = {}
    for idx, op in enumerate(sched.ops):
        for r in _sources(op):
            last_use[r] = idx
    for r in sched.outputs:
        last_use[r] = len(sched.ops)
    reg = {i: cts[i] for i in range(sched.n_inputs)}
    N, t = sched.N, ctx.t
    pt_cache = {}

    def plain(slots):
        key = id(slots)
        if key not in pt_cache:
            pt_cache[key] = bfv.encode(ctx, dense_slots(slots, N, t))
        return pt_cache[key]

    for idx, op in enumerate(sched.ops):
        k = op[0]
        if k == "mul_scalar":
            reg[op[1]] = bfv.mul_scalar(ctx, reg[op[2]], op[3])
        elif k == "add":
            reg[op[1]] = bfv.add(ctx, reg[op[2]], reg[op[3]])
        elif k == "add_plain":
            reg[op[1]] = bfv.add_plain(ctx, reg[op[2]], plain(op[3]))
        elif k == "mul_plain":
            reg[op[1]] = bfv.mul_plain(ctx, reg[op[2]], plain(op[3]))
        elif k == "rotate":
            reg[op[1]] = bfv.rotate(ctx, reg[op[2]], op[3], keys)
        elif k == "rotate_hoisted":
            reg[op[1]] = bfv.rotate_hoisted(ctx, reg[op[2]], op[3], keys)
        elif k == "square":
            reg[op[1]] = bfv.square(ctx, reg[op[2]], keys)
        else:
            raise ValueError(k)
        if not keep:
            for r in _sources(op):
                if last_use.get(r) == idx and r not in sched.outputs:
                    reg.pop(r, None)
        if progress is not None and (idx + 1) % 250 == 0:
            progress(idx + 1, len(sched.ops))
    return [reg[o] for o in sched.outputs], reg
