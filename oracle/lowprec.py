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


def store_links(U, fmt, link=18):
    """Round links to the storage format (links are never scaled: |U_ij| <= 1).

    ``link=12`` emulates the two-row storage: rows 0 and 1 are rounded and
    row 2 is rebuilt from the rounded rows (``third_row``, evaluated in
    float64), as the library does in registers."""
    R = _round_links(U, fmt)
    if link == 18:
        return R
    if link != 12:
        raise ValueError(f"link must be 18 or 12, got {link!r}")
    out = R.copy()
    out[..., 2, :] = third_row(R)
    return out
