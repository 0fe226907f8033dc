"""Counter-based random numbers for the stochastic stress (oracle side).

TEST INFRASTRUCTURE ONLY: this package is the plain FP64 CPU oracle that the
HIP path is checked against. Only tests, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path never does.

The paper asks for i.i.d. unit normal variates W^n regenerated every time step
(Sec. III.B.2, definition of the stochastic flux Sigma^n) but does not say how
they are drawn. Both sides of the parity check draw them from one
counter-based generator, Philox4x32 with 10 rounds, implemented here from its
published definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11), and turn uniforms into normals with the
Box-Muller transform (Box & Muller, 1958).

Counter and key layout (a convention of this project, shared with the GPU):
  key     = (seed mod 2^32, seed >> 32)
  counter = (index, step mod 2^32, (replica << 4) | block, step >> 32)
For the stochastic stress of a step, the two cells (i, j, 2m) and
(i, j, 2m+1) share index i + Nx*(j + Ny*m) and blocks 0, 1, 2: twelve words
for their twelve normals. Block 3, with index i + Nx*(j + Ny*k) per cell,
draws the optional equilibrium initial velocity.

Parity unpinned: no known-answer vectors are available to this project, so the
exact words are checked only by the two independent implementations agreeing
bit for bit, by a big-integer re-statement of the round function in the tests,
and by statistical tests of the uniforms and normals.
"""
import numpy as np

# Round multipliers and Weyl key increments of Philox4x32 (Salmon et al. 2011).
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 bijection of a 128-bit counter under a 64-bit key.

    Every argument is an unsigned 32-bit integer or array (broadcast). One round
    multiplies words 0 and 2 by fixed odd constants, forms the 64-bit
    products' high and low halves, and mixes them with the other two words and
    the round key; the key is bumped by the Weyl constants between rounds.
    Returns four uint32 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    k0 = int(k0) & MASK32
    k1 = int(k1) & MASK32
    m = np.uint64(MASK32)
    sh = np.uint64(32)
    for _ in range(10):
        p0 = np.uint64(PHILOX_M0) * c0
        p1 = np.uint64(PHILOX_M1) * c2
        hi0, lo0 = p0 >> sh, p0 & m
        hi1, lo1 = p1 >> sh, p1 & m
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + PHILOX_W0) & MASK32
        k1 = (k1 + PHILOX_W1) & MASK32
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def uniform_open0(w):
    """Word -> uniform in (0, 1]: (w + 1) * 2^-32 (never zero, safe for log)."""
    return (w.astype(np.float64) + 1.0) * 2.0 ** -32


def uniform_closed0(w):
    """Word -> uniform in [0, 1): w * 2^-32."""
    return w.astype(np.float64) * 2.0 ** -32


def box_muller(wa, wb):
    """Two words -> two independent standard normals (Box-Muller, 1958).

    The first word gives the radius through -2 ln u1 with u1 in (0,1], the
    second the angle 2 pi u2 with u2 in [0,1).
    """
    u1 = uniform_open0(wa)
    u2 = uniform_closed0(wb)
    r = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return r * np.cos(ang), r * np.sin(ang)


def cell_words(n_cells, step, seed, replica, block):
    """The four Philox words of `block` for every counter index 0..n_cells-1."""
    cells = np.arange(n_cells, dtype=np.uint64)
    step = int(step)
    seed = int(seed)
    return philox4x32_10(cells, step & MASK32,
                         ((int(replica) << 4) | int(block)) & MASK32,
                         (step >> 32) & MASK32,
                         seed & MASK32, (seed >> 32) & MASK32)


def stress_normals(n, step, seed, replica):
    """Six unit normals per cell for the symmetric stochastic stress on an
    Nx x Ny x Nz grid (Nz even).

    Cells (i, j, 2m) (lower) and (i, j, 2m+1) (upper) share the counter index
    i + Nx*(j + Ny*m). With A, B, C the words of blocks 0, 1, 2:
      lower: (A0,A1) -> (W_xx, W_yy), (A2,A3) -> (W_zz, W_xy), (B0,B1) -> (W_xz, W_yz)
      upper: (B2,B3) -> (W_xx, W_yy), (C0,C1) -> (W_zz, W_xy), (C2,C3) -> (W_xz, W_yz)
    Returns a dict of flat float64 arrays indexed by cell i + Nx*(j + Ny*k).
    """
    nx, ny, nz = (int(x) for x in n)
    if nz % 2:
        raise ValueError("the paired stress stream needs an even Nz (got %d)" % nz)
    npairs = nx * ny * (nz // 2)
    A = cell_words(npairs, step, seed, replica, 0)
    B = cell_words(npairs, step, seed, replica, 1)
    C = cell_words(npairs, step, seed, replica, 2)
    lower, upper = {}, {}
    lower["xx"], lower["yy"] = box_muller(A[0], A[1])
    lower["zz"], lower["xy"] = box_muller(A[2], A[3])
    lower["xz"], lower["yz"] = box_muller(B[0], B[1])
    upper["xx"], upper["yy"] = box_muller(B[2], B[3])
    upper["zz"], upper["xy"] = box_muller(C[0], C[1])
    upper["xz"], upper["yz"] = box_muller(C[2], C[3])
    out = {}
    for key in ("xx", "yy", "zz", "xy", "xz", "yz"):
        w = np.empty((nz // 2, 2, ny * nx))
        w[:, 0, :] = lower[key].reshape(nz // 2, ny * nx)
        w[:, 1, :] = upper[key].reshape(nz // 2, ny * nx)
        out[key] = w.reshape(-1)
    return out


def equilibrium_normals(n_cells, seed, replica):
    """Three unit normals per cell (one per face family) from block 3.

    Words (w0,w1) -> (x-face, y-face), (w2,w3) -> (z-face, unused).
    """
    a0, a1, a2, a3 = cell_words(n_cells, 0, seed, replica, 3)
    nx_, ny_ = box_muller(a0, a1)
    nz_, _ = box_muller(a2, a3)
    return nx_, ny_, nz_
