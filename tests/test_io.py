"""Storage reads and writes of the chunk pipeline (tp_io_*; paper, Section 2.3:
chunks read from and written to the storage drive by their own threads).
Host code only: these run on the CPU."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def tp():
    from paper_2209_08450_amd import tp as mod
    return mod


def _aligned_empty(shape, dtype, align=4096):
    n = int(np.prod(shape)) * np.dtype(dtype).itemsize
    raw = np.empty(n + align, np.uint8)
    off = (-raw.ctypes.data) % align
    return raw[off:off + n].view(dtype).reshape(shape)


@pytest.mark.parametrize("threads", [1, 3, 16])
def test_read_rows_matches_slicing(tp, tmp_path, threads):
    rng = np.random.default_rng(1)
    a = rng.integers(0, 4096, (7, 13, 10)).astype(np.uint16)  # [angles][rows][cols]
    p = tmp_path / "proj.raw"
    a.tofile(p)
    for z0, z1 in [(0, 13), (2, 5), (12, 13)]:
        dst = np.empty((7, z1 - z0, 10), np.uint16)
        tp.io_read_rows(p, 7, 13, 10, z0, z1, dst, threads=threads)
        assert np.array_equal(dst, a[:, z0:z1])


def test_read_rows_with_header_and_float(tp, tmp_path):
    rng = np.random.default_rng(2)
    a = rng.standard_normal((3, 6, 5)).astype(np.float32)
    p = tmp_path / "f.raw"
    with open(p, "wb") as f:
        f.write(b"H" * 100)
        f.write(a.tobytes())
    dst = np.empty((3, 2, 5), np.float32)
    tp.io_read_rows(p, 3, 6, 5, 1, 3, dst, header_bytes=100, elem_bytes=4)
    assert np.array_equal(dst, a[:, 1:3])


def test_aligned_read_and_write_round_trip(tp, tmp_path):
    # 2048 columns of uint16 and 4096-byte aligned buffers: every piece is
    # aligned, so the calls open the files for direct I/O where the file
    # system allows it (else buffered); the bytes are the same either way
    rng = np.random.default_rng(3)
    a = rng.integers(0, 65535, (4, 8, 2048)).astype(np.uint16)
    p = tmp_path / "aligned.raw"
    a.tofile(p)
    dst = _aligned_empty((4, 4, 2048), np.uint16)
    tp.io_read_rows(p, 4, 8, 2048, 2, 6, dst, threads=4)
    assert np.array_equal(dst, a[:, 2:6])
    vol = _aligned_empty((6, 32, 32), np.float32)
    vol[:] = rng.standard_normal(vol.shape)
    q = tmp_path / "vol.raw"
    tp.io_create(q, 10 * 32 * 32 * 4)
    tp.io_write_slices(q, 3, vol, 32 * 32 * 4, threads=3)
    back = np.fromfile(q, np.float32).reshape(10, 32, 32)
    assert np.array_equal(back[3:9], vol)
    assert not back[:3].any() and not back[9:].any()


def test_write_slices_in_any_order(tp, tmp_path):
    rng = np.random.default_rng(4)
    vol = rng.standard_normal((9, 5, 5)).astype(np.float32)
    q = tmp_path / "v.raw"
    tp.io_create(q, vol.nbytes)
    for z0, z1 in [(6, 9), (0, 2), (2, 6)]:
        tp.io_write_slices(q, z0, vol[z0:z1], 5 * 5 * 4, threads=2)
    assert np.array_equal(np.fromfile(q, np.float32).reshape(9, 5, 5), vol)


def test_io_errors(tp, tmp_path):
    dst = np.empty((2, 2, 4), np.uint16)
    with pytest.raises(tp.TpError, match="cannot open"):
        tp.io_read_rows(tmp_path / "missing.raw", 2, 4, 4, 0, 2, dst)
    p = tmp_path / "short.raw"
    np.zeros(10, np.uint16).tofile(p)
    with pytest.raises(tp.TpError, match="too short"):
        tp.io_read_rows(p, 2, 4, 4, 0, 2, dst)
    with pytest.raises(tp.TpError, match="row range"):
        tp.io_read_rows(p, 2, 4, 4, 3, 5, dst)
    with pytest.raises(ValueError):
        tp.io_read_rows(p, 2, 4, 4, 0, 2, np.empty(3, np.uint16))
    with pytest.raises(tp.TpError, match="cannot open"):
        tp.io_write_slices(tmp_path / "nodir" / "x.raw", 0, np.zeros(4, np.float32), 16)
    assert tp._io_read_rows(None, 0, 1, 1, 1, 0, 1, 2, None, 1) == tp.TP_EINVAL
