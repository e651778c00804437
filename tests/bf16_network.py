"""A hand-built 65-64-64-1 network whose bfloat16 inference logit is known
exactly, for pinning the BF16 emulation of the oracle (and, through it, the
GPU kernel).

Eight disjoint paths, each through its own input and hidden units, add up in
the logit.  Every value on a path is a short binary fraction, so every
float32 sum and product below is exact and the only effect of each rounding
site (input, W1, h1, W2, h2, W3) and of each bias is the one worked out by
hand here.  bfloat16 keeps 8 significant bits: near 1 its spacing is 2^-7,
so 1 + 3*2^-9 rounds up to 1 + 2^-7 and -(1 - 2^-12) rounds to -1.

  path  what it tests     value on the path (correct emulation)       logit term
  0     x rounded         x = 1 + 3*2^-9 -> 1 + 2^-7; a1 = x - 1      2^-7
  1     W1 rounded        W1 = 1 + 3*2^-9 -> 1 + 2^-7; a1 = W1 - 1    2^-7
  2     b1 kept exact     a1 = 1 + (-(1 - 2^-12)) = 2^-12             2^-12
  3     h1 rounded        a1 = 1 + 3*2^-9 -> h1 = 1 + 2^-7; a2 = h1-1 2^-7
  4     W2 rounded        W2 = 1 + 3*2^-9 -> 1 + 2^-7; a2 = W2 - 1    2^-7
  5     b2 kept exact     a2 = 1 + (-(1 - 2^-12)) = 2^-12             2^-12
  6     h2 rounded        a2 = 1 + 3*2^-9 -> h2 = 1 + 2^-7           1 + 2^-7
  7     W3 rounded        W3 = 1 + 3*2^-9 -> 1 + 2^-7 (h2 = 1)        1 + 2^-7
  out   b3 kept exact     b3 = -(1 - 2^-12)                           -1 + 2^-12

Sum: 4*2^-7 + 2*2^-12 + 2*(1 + 2^-7) - 1 + 2^-12 = 1 + 6*2^-7 + 3*2^-12.
Leaving out one rounding site moves one path term by -2^-9 (the unrounded
1 + 3*2^-9 instead of 1 + 2^-7, or 1.5*2^-8 instead of 2^-7); rounding one
bias moves a 2^-12 term to 0.  Ties do not occur on any path.
"""
import numpy as np

NI, NH = 65, 64
EXPECTED_LOGIT = 1.0 + 6 * 2.0**-7 + 3 * 2.0**-12
UP = 1.0 + 3 * 2.0**-9          # rounds up to 1 + 2^-7 in bfloat16
JUST_UNDER_ONE = 1.0 - 2.0**-12  # rounds to 1 in bfloat16


def network():
    """(params[8449] float32, X[1][65] float32)."""
    W1 = np.zeros((NH, NI), np.float32)
    b1 = np.zeros(NH, np.float32)
    W2 = np.zeros((NH, NH), np.float32)
    b2 = np.zeros(NH, np.float32)
    W3 = np.zeros(NH, np.float32)
    x = np.zeros(NI, np.float32)
    for u in range(8):           # input u feeds hidden unit u, which feeds unit u
        x[u] = 1.0
        W1[u, u] = 1.0
        W2[u, u] = 1.0
        W3[u] = 1.0
    x[0] = UP                    # path 0
    b1[0] = -1.0
    W1[1, 1] = UP                # path 1
    b1[1] = -1.0
    b1[2] = -JUST_UNDER_ONE      # path 2
    b1[3] = 3 * 2.0**-9          # path 3 (bfloat16-exact bias)
    b2[3] = -1.0
    W2[4, 4] = UP                # path 4
    b2[4] = -1.0
    b2[5] = -JUST_UNDER_ONE      # path 5
    b2[6] = 3 * 2.0**-9          # path 6
    W3[7] = UP                   # path 7
    b3 = np.array([-JUST_UNDER_ONE], np.float32)
    params = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, b3]).astype(np.float32)
    assert params.size == 8449
    return params, x[None, :]
