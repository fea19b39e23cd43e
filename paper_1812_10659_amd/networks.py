"""Client-side helpers around compiled plans: the layer lists of the three
network shapes, packing input values into slot vectors with a plan's input
map, and reading results with its output map.  Pure indexing: every
homomorphic step runs in the library."""
from __future__ import annotations

import numpy as np

from . import lola
from . import workloads as wl

# The 28x28 image is zero-padded to 29x29 (one row at the bottom, one column
# at the right) so that 13 windows of 5 at stride 2 cover it.
MNIST_PAD = 29


def mnist_layers(w: wl.MnistWeights):
    return [lola.conv2d(w.conv_w, w.conv_b, MNIST_PAD, 2), lola.square(),
            lola.dense(w.w1, w.b1), lola.square(), lola.dense(w.w2, w.b2)]


def mnist_dense_layers(w: wl.MnistWeights):
    """LoLa-Dense: the MNIST-shaped network with the image sent as one dense
    message (padded 29 x 29, row by row; values from mnist_input_values)."""
    return [lola.conv2d(w.conv_w, w.conv_b, MNIST_PAD, 2, dense_input=True), lola.square(),
            lola.dense(w.w1, w.b1), lola.square(), lola.dense(w.w2, w.b2)]


def cifar_layers(w: wl.CifarWeights, n_in: int = 34):
    """The collapsed CIFAR network on a padded n_in x n_in input: 8x8
    convolution over 3 channels at stride 2, square, 6x6 convolution over
    all maps at stride 2, square, dense -> 10."""
    n1 = (n_in - w.conv1_w.shape[-1]) // 2 + 1
    return [lola.conv2d(w.conv1_w, w.conv1_b, n_in, 2), lola.square(),
            lola.conv2d(w.conv2_w, w.conv2_b, n1, 2), lola.square(), lola.dense(w.w3, w.b3)]


def cifar_input_values(img) -> np.ndarray:
    """The [3][H][W] image zero-padded by one pixel on every side, flattened
    channel by channel, row by row."""
    img = np.asarray(img, dtype=np.int64)
    c, h, w = img.shape
    p = np.zeros((c, h + 2, w + 2), dtype=np.int64)
    p[:, 1:h + 1, 1:w + 1] = img
    return p.reshape(-1)


def mnist_small_layers(w: wl.MnistSmallWeights):
    """The small variant: convolution, square, one dense layer 845 -> 10."""
    return [lola.conv2d(w.conv_w, w.conv_b, MNIST_PAD, 2), lola.square(), lola.dense(w.w, w.b)]


def mnist_input_values(img) -> np.ndarray:
    p = np.zeros((MNIST_PAD, MNIST_PAD), dtype=np.int64)
    p[:28, :28] = img
    return p.reshape(-1)


def dense64_layers(W):
    return [lola.dense(W), lola.square()]


def head_layers(w: wl.HeadWeights, n_hidden: int | None = None):
    nh = w.w1.shape[0] if n_hidden is None else n_hidden
    return [lola.dense(w.w1[:nh], w.b1[:nh]), lola.square(), lola.dense(w.w2[:, :nh], w.b2)]


def pack_inputs(input_map: np.ndarray, values: np.ndarray) -> np.ndarray:
    """Slot vectors [n_inputs][N]: slot s of message m holds values[map[m, s]]
    (0 where the map is -1)."""
    v = np.asarray(values, dtype=np.int64).reshape(-1)
    out = np.zeros(input_map.shape, dtype=np.int64)
    sel = input_map >= 0
    out[sel] = v[input_map[sel]]
    return out


def unpack_outputs(output_map: np.ndarray, slots) -> np.ndarray:
    """Result values from the decoded output messages (slots [n_outputs][N])."""
    s = np.asarray(slots)
    n = int(output_map.max()) + 1
    res = np.zeros(n, dtype=np.int64)
    sel = output_map >= 0
    res[output_map[sel]] = s[sel]
    return res
