"""Standard Gaussian draws from Philox words (Omega of Alg. 3 step 1 / Alg. 4 step 1).

The paper asks for an n x l matrix of i.i.d. N(0, 1) entries (Sec. III). The
reading used here, and written out independently on the device, is:

  * element e of Omega (column-major, e = i + j*n) uses the Philox4x64-10 block
    with counter (e // 4, 0, word2, 0) and key (seed, stream); it takes normal
    number e % 4 of that block. Column-major numbering nests in l: the first l
    columns of an n x l' draw equal the n x l draw.
  * each 64-bit word w becomes u = (w >> 12) * 2^-52 + 2^-53, an exact dyadic in
    (0, 1).
  * Box-Muller on (u0, u1) and (u2, u3):  r = sqrt(-2 log u_even),
    t = 2 pi u_odd,  (z_even, z_odd) = (r cos t, r sin t).
  * log, sin and cos are computed by the fixed sequences of IEEE-754 double
    operations below (+, -, *, / and sqrt, each rounded once, no fused
    multiply-add). Any implementation that performs the same sequence gets
    the same bits, which is what makes host and device Omega identical.

    log u:  u = f * 2^e with f in (sqrt(1/2), sqrt(2)] (exact, from the bits);
            s = (f - 1) / (f + 1);  z = s * s;
            p = 1/23;  p = 1/(2j+1) + z * p  for j = 10, 9, ..., 0;
            log u = e * LN2 + (2 * s) * p,   LN2 = 0.6931471805599453.
    sin/cos of 2 pi u with u = (2t + 1) * 2^-53:
            quadrant qd = (2t + 1 + 2^50) >> 51 (= round(4u), integer exact);
            f = ((2t + 1) - qd * 2^51) * 2^-51 in [-1/2, 1/2) (exact);
            x = f * PIO2, PIO2 = 1.5707963267948966;  z = x * x;
            S = 1;  S = 1 - (z * S) / ((2j)(2j+1))  for j = 10, ..., 1;  sin x = x * S;
            C = 1;  C = 1 - (z * C) / ((2j-1)(2j))  for j = 10, ..., 1;  cos x = C;
            rotate (sin x, cos x) by qd quarter turns.

Test infrastructure only (see ``oracle/__init__``).
"""
import numpy as np

from .philox import block_words

LN2 = 0.6931471805599453
PIO2 = 1.5707963267948966
SQRT2 = 1.4142135623730951


def uniform_from_words(w):
    """Map uint64 words to exact dyadic uniforms (w >> 12) * 2^-52 + 2^-53 in (0, 1)."""
    w = np.asarray(w, dtype=np.uint64)
    t = (w >> np.uint64(12)).astype(np.float64)  # < 2^52, exact
    return t * 2.0 ** -52 + 2.0 ** -53            # exact: 53 significant bits


def own_log(u):
    """Natural log of u in (0, 1] by the fixed operation sequence in the module doc."""
    u = np.asarray(u, dtype=np.float64)
    f, e = np.frexp(u)                 # u = f * 2^e, f in [1/2, 1), exact
    f = f * 2.0                        # f in [1, 2), exact
    e = e - 1
    big = f > SQRT2
    f = np.where(big, f * 0.5, f)      # f in (sqrt(1/2), sqrt(2)], exact
    e = np.where(big, e + 1, e).astype(np.float64)
    s = (f - 1.0) / (f + 1.0)
    z = s * s
    p = np.full_like(z, 1.0 / 23.0)
    for j in range(10, -1, -1):
        p = 1.0 / (2 * j + 1) + z * p
    return e * LN2 + (2.0 * s) * p


def own_sincos_2pi(w):
    """(sin, cos) of 2*pi*u for u = uniform_from_words(w), by the module-doc sequence."""
    w = np.asarray(w, dtype=np.uint64)
    t = (w >> np.uint64(12)).astype(np.int64)           # u = (2t+1) * 2^-53
    odd = 2 * t + 1                                     # < 2^53
    qd = (odd + (1 << 50)) >> 51                        # round(4u), 0..4
    f = (odd - qd * (1 << 51)).astype(np.float64) * 2.0 ** -51
    x = f * PIO2
    z = x * x
    S = np.ones_like(z)
    C = np.ones_like(z)
    for j in range(10, 0, -1):
        S = 1.0 - (z * S) / float((2 * j) * (2 * j + 1))
        C = 1.0 - (z * C) / float((2 * j - 1) * (2 * j))
    sx = x * S
    cx = C
    qm = qd & 3
    sin_t = np.select([qm == 0, qm == 1, qm == 2, qm == 3], [sx, cx, -sx, -cx])
    cos_t = np.select([qm == 0, qm == 1, qm == 2, qm == 3], [cx, -sx, -cx, sx])
    return sin_t, cos_t


def normals_from_block(words):
    """Four N(0,1) numbers from one Philox block (..., 4) of uint64 words."""
    u0 = uniform_from_words(words[..., 0])
    u2 = uniform_from_words(words[..., 2])
    r01 = np.sqrt(-2.0 * own_log(u0))
    r23 = np.sqrt(-2.0 * own_log(u2))
    s01, c01 = own_sincos_2pi(words[..., 1])
    s23, c23 = own_sincos_2pi(words[..., 3])
    return np.stack([r01 * c01, r01 * s01, r23 * c23, r23 * s23], axis=-1)


def gaussian_matrix(seed, rows, cols, stream=0, word2=0):
    """rows x cols matrix of N(0,1) draws, element (i, j) = normal number i + j*rows."""
    count = rows * cols
    if count == 0:
        return np.zeros((rows, cols))
    nblk = (count + 3) // 4
    z = normals_from_block(block_words(seed, stream, np.arange(nblk, dtype=np.uint64), word2))
    flat = z.reshape(-1)[:count]
    return flat.reshape(cols, rows).T.copy()
