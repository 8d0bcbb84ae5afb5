"""Storage-precision emulation for the mixed-precision solve of Algorithm 1.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's solver keeps the outer loop in high precision and runs the inner
CG "mainly in low precision" (Kernel Description).  To check that the
Algorithm 1 reading converges with the low-precision formats the GPU uses,
vectors are rounded to those formats after each step:

* ``"f64"``  -- no rounding;
* ``"f32"``  -- every complex component rounded to IEEE binary32;
* ``"f16s"`` -- per-site scaled binary16: s(n) = max over the 24 reals of the
                site, stored as binary32; payload = binary16(v / s(n)) with
                round-to-nearest-even, so every stored component is in [-1, 1];
* ``"bf16s"`` -- the same with bfloat16 payloads (round-to-nearest-even).

Links are stored unscaled in the same formats, as the full matrix, as its
first two rows (12 reals, row 2 rebuilt), or in the 10-real form
(``pack10``: row 0 and two entries of a pivot column).
"""

import numpy as np

FORMATS = ("f64", "f32", "f16s", "bf16s")


def _round_bf16(x):
    """float64 -> nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def site_scale(v):
    """Per-site scale s(n) = max |real component| over spin and colour, as binary32."""
    re = np.abs(np.real(v))
    im = np.abs(np.imag(v))
    m = np.maximum(re.max(axis=(-1, -2)), im.max(axis=(-1, -2)))
    return m.astype(np.float32).astype(np.float64)


def store(v, fmt):
    """Round a canonical spinor field to the storage format ``fmt``."""
    v = np.asarray(v, dtype=np.complex128)
    if fmt == "f64":
        return v
    if fmt == "f32":
        return v.astype(np.complex64).astype(np.complex128)
    if fmt in ("f16s", "bf16s"):
        s = site_scale(v)
        safe = np.where(s > 0, s, 1.0)[..., None, None]
        re = np.real(v) / safe
        im = np.imag(v) / safe
        if fmt == "f16s":
            re = re.astype(np.float16).astype(np.float64)
            im = im.astype(np.float16).astype(np.float64)
        else:
            re = _round_bf16(re)
            im = _round_bf16(im)
        return (re + 1j * im) * safe
    raise ValueError(f"unknown format {fmt!r}")


def _round_links(U, fmt):
    U = np.asarray(U, dtype=np.complex128)
    if fmt == "f64":
        return U
    if fmt == "f32":
        return U.astype(np.complex64).astype(np.complex128)
    if fmt == "f16s":
        return (np.real(U).astype(np.float16).astype(np.float64)
                + 1j * np.imag(U).astype(np.float16).astype(np.float64))
    if fmt == "bf16s":
        return _round_bf16(np.real(U)) + 1j * _round_bf16(np.imag(U))
    raise ValueError(f"unknown format {fmt!r}")


def third_row(U):
    """Row 2 of an SU(3) matrix from its rows 0 and 1.

    For a special unitary matrix the rows form a right-handed orthonormal
    basis of C^3: each row is the complex conjugate of the cross product of
    the other two (unitarity gives orthogonality, det = 1 fixes the phase).
    So row 2 = conj(row 0 x row 1)."""
    a = U[..., 0, :]
    b = U[..., 1, :]
    return np.conj(np.cross(a, b))


def _round_reals(x, fmt):
    x = np.asarray(x, dtype=np.float64)
    if fmt == "f64":
        return x
    if fmt == "f32":
        return x.astype(np.float32).astype(np.float64)
    if fmt == "f16s":
        return x.astype(np.float16).astype(np.float64)
    if fmt == "bf16s":
        return _round_bf16(x)
    raise ValueError(f"unknown format {fmt!r}")


def pack8(U, pivot=True):
    """The 8-real form of SU(3) links (one more byte per link for the pivot).

    For a special unitary U, row 0 and column 0 are unit vectors and every
    entry is the complex conjugate of its cofactor, so the four entries
    outside row 0 and column 0 follow from U_01, U_02, U_10 and the phases of
    U_00 and U_20 (the moduli from unit norm).  The rebuild divides by
    N = 1 - |U_00|^2 = |U_01|^2 + |U_02|^2, which vanishes for the identity.
    So the columns are first rotated cyclically (a determinant-one
    permutation, V = U P stays special unitary) to bring the column k whose
    row-0 entry has the smallest modulus to the front: then |V_00|^2 <= 1/3
    and N >= 2/3 for every link.  ``pivot=False`` keeps k = 0 (for tests).

    Returns (k, reals) with reals[..., :] = (Re V01, Im V01, Re V02, Im V02,
    Re V10, Im V10, arg V00 / 2 pi, arg V20 / 2 pi); phases in revolutions."""
    U = np.asarray(U, dtype=np.complex128)
    row0 = U[..., 0, :]
    if pivot:
        k = np.argmin(row0.real ** 2 + row0.imag ** 2, axis=-1)
    else:
        k = np.zeros(U.shape[:-2], dtype=np.int64)
    cols = (k[..., None] + np.arange(3)) % 3
    V = np.take_along_axis(U, np.broadcast_to(cols[..., None, :], U.shape), axis=-1)
    reals = np.stack([V[..., 0, 1].real, V[..., 0, 1].imag, V[..., 0, 2].real, V[..., 0, 2].imag,
                      V[..., 1, 0].real, V[..., 1, 0].imag,
                      np.angle(V[..., 0, 0]) / (2 * np.pi), np.angle(V[..., 2, 0]) / (2 * np.pi)], axis=-1)
    return k, reals


def unpack8(k, reals):
    """The link matrices of the 8-real form (inverse of ``pack8``), in float64."""
    r = np.asarray(reals, dtype=np.float64)
    a1 = r[..., 0] + 1j * r[..., 1]
    a2 = r[..., 2] + 1j * r[..., 3]
    b0 = r[..., 4] + 1j * r[..., 5]
    n = np.abs(a1) ** 2 + np.abs(a2) ** 2            # 1 - |a0|^2
    a0 = np.sqrt(np.maximum(1.0 - n, 0.0)) * np.exp(2j * np.pi * r[..., 6])
    c0 = np.sqrt(np.maximum(n - np.abs(b0) ** 2, 0.0)) * np.exp(2j * np.pi * r[..., 7])
    # conj(U_ij) = cofactor_ij, solved for the entries outside row 0 and column 0
    b1 = -(np.conj(a0) * a1 * b0 + np.conj(a2) * np.conj(c0)) / n
    b2 = (np.conj(a1) * np.conj(c0) - np.conj(a0) * a2 * b0) / n
    c1 = np.conj(a2) * np.conj(b0) - np.conj(a0) * np.conj(b2)
    c2 = np.conj(a0) * np.conj(b1) - np.conj(a1) * np.conj(b0)
    V = np.stack([np.stack([a0, a1, a2], -1), np.stack([b0, b1, b2], -1), np.stack([c0, c1, c2], -1)], -2)
    k = np.asarray(k)
    cols = (np.arange(3) - k[..., None]) % 3       # undo the cyclic rotation
    return np.take_along_axis(V, np.broadcast_to(cols[..., None, :], V.shape), axis=-1)


def _abs2(z):
    return z.real * z.real + z.imag * z.imag


def pack10(U, fmt="f64"):
    """The 10-real form of SU(3) links: row 0 and, for the pivot column k,
    the entries of rows 1 and 2, each rounded to the storage format.

    The pivot is the column whose row-0 entry has the smallest modulus as
    stored (the lowest index on ties), so it can be found again from the
    stored row; the rebuild (``unpack10``) then divides by
    N = |U_0,k+1|^2 + |U_0,k+2|^2 >= 2/3 and derives no modulus by
    cancellation, and needs no trigonometric function.

    Returns (row0 [..., 3] complex, k [...], col [..., 2] complex)."""
    U = np.asarray(U, dtype=np.complex128)
    row0 = _round_reals(U[..., 0, :].real, fmt) + 1j * _round_reals(U[..., 0, :].imag, fmt)
    k = np.argmin(_abs2(row0), axis=-1)
    col = np.take_along_axis(U[..., 1:, :], np.broadcast_to(k[..., None, None], U.shape[:-2] + (2, 1)),
                             axis=-1)[..., 0]
    col = _round_reals(col.real, fmt) + 1j * _round_reals(col.imag, fmt)
    return row0, k, col


def unpack10(row0, k, col):
    """The link matrices of the 10-real form (inverse of ``pack10``), in
    float64.  With V = U P (the columns rotated cyclically so that the pivot
    comes first, still special unitary) the entries of V outside row 0 and
    column 0 follow from conj(V_ij) = cofactor_ij."""
    k = np.asarray(k)
    sel = lambda j: np.take_along_axis(row0, ((k + j) % 3)[..., None], axis=-1)[..., 0]  # noqa: E731
    a0, a1, a2 = sel(0), sel(1), sel(2)
    b0, c0 = col[..., 0], col[..., 1]
    n = _abs2(a1) + _abs2(a2)
    b1 = -(np.conj(a0) * a1 * b0 + np.conj(a2) * np.conj(c0)) / n
    b2 = (np.conj(a1) * np.conj(c0) - np.conj(a0) * a2 * b0) / n
    c1 = np.conj(a2) * np.conj(b0) - np.conj(a0) * np.conj(b2)
    c2 = np.conj(a0) * np.conj(b1) - np.conj(a1) * np.conj(b0)
    out = np.empty(row0.shape[:-1] + (3, 3), dtype=np.complex128)
    out[..., 0, :] = row0
    for j, (b, c) in enumerate(((b0, c0), (b1, c1), (b2, c2))):
        cols = ((k + j) % 3)[..., None]
        np.put_along_axis(out[..., 1, :], cols, b[..., None], axis=-1)
        np.put_along_axis(out[..., 2, :], cols, c[..., None], axis=-1)
    return out


def store_links(U, fmt, link=18, pivot=True):
    """Round links to the storage format (links are never scaled: |U_ij| <= 1).

    ``link=12`` emulates the two-row storage: rows 0 and 1 are rounded and
    row 2 is rebuilt from the rounded rows (``third_row``, evaluated in
    float64), as the library does in registers.  ``link=10`` emulates the
    10-real form (``pack10``), ``link=8`` the 8-real form (``pack8``, not
    used by the library: see its tests): the reals are rounded to the format
    and the matrix rebuilt from them in float64."""
    if link == 8:
        k, reals = pack8(U, pivot)
        return unpack8(k, _round_reals(reals, fmt))
    if link == 10:
        return unpack10(*pack10(U, fmt))
    R = _round_links(U, fmt)
    if link == 18:
        return R
    if link != 12:
        raise ValueError(f"link must be 18, 12, 10 or 8, got {link!r}")
    out = R.copy()
    out[..., 2, :] = third_row(R)
    return out
