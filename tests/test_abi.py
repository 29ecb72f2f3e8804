"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function that include/scdrop.h declares, and rejects bad parameters
before touching the device."""
import ctypes

import pytest

import paper_0910_3915_amd as scd
from paper_0910_3915_amd import binding as B
import workloads as W


def test_library_exports_header_symbols():
    L = scd.lib()
    names = scd.header_symbols()
    assert len(names) >= 30
    for n in names:
        assert hasattr(L, n), n
    assert b"gfx950" in L.scd_version()


def test_struct_layouts_match_header():
    # sizes implied by the header's field lists (natural alignment)
    assert ctypes.sizeof(B.ScdParams) == 6 * 4 + 9 * 8
    assert ctypes.sizeof(B.ScdObs) == 5 * 8 + 2 * 4 + 8
    assert ctypes.sizeof(B.ScdCaCfg) == 4 * 4 + 8
    assert ctypes.sizeof(B.ScdCa) == 14 * 8 + 2 * 4


def _sizes(p):
    sp = B.make_params(p)
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    return scd.lib().scd_sizes(ctypes.byref(sp), ctypes.byref(a), ctypes.byref(b)), a.value, b.value


def test_sizes_and_validation():
    st, pop, work = _sizes(W.params(32, 32, 32, 0.1))
    assert st == 0 and pop == 2 * 19 * 32 ** 3 * 8 and work > 32 ** 3 * 4
    st, pop32, _ = _sizes(W.params(32, 32, 32, 0.1, dtype="f32"))
    assert st == 0 and pop32 == pop // 2
    bad = [W.params(32, 32, 32, 0.1, tau=(0.5, 1.0)),
           W.params(0, 32, 32, 0.1),
           W.params(32, 32, 32, -0.1),
           W.params(32, 32, 32, 0.1, rho_wall=(-0.1, 0.5)),
           W.params(32, 32, 32, 0.1, g_wall=(0.1, float("nan"))),
           dict(W.params(32, 32, 32, 0.1), psi=3)]
    for p in bad:
        st, _, _ = _sizes(p)
        assert st == B.SCD_EINVAL, p
        assert scd.lib().scd_last_error()


def test_pop_buffer_is_blocked_with_padded_planes():
    """Population buffers hold 2 species x nz planes x ceil(nx ny / 32)
    blocks x 19 velocities x 32 slots; the per-species 4 GiB bound of the
    32-bit offsets counts the padded slots."""
    for (nx, ny, nz) in ((20, 18, 14), (7, 5, 3), (33, 1, 2)):
        st, pop, _ = _sizes(W.params(nx, ny, nz, 0.1))
        assert st == 0
        assert pop == 2 * 19 * 32 * ((nx * ny + 31) // 32) * nz * 8, (nx, ny, nz)
    assert _sizes(W.params(256, 256, 256, 0.1))[0] == 0          # 2.55 GB per species
    st, _, _ = _sizes(W.params(320, 320, 320, 0.1))
    assert st == B.SCD_EUNSUPPORTED                              # 4.98 GB per species
    assert _sizes(W.params(320, 320, 320, 0.1, dtype="f32"))[0] == 0


def test_adjoint_flag_grows_work_area():
    p = W.params(16, 16, 12, 0.1)
    sp0, sp1 = B.make_params(p), B.make_params(p, adjoint=True)
    a, w0, w1 = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    scd.lib().scd_sizes(ctypes.byref(sp0), ctypes.byref(a), ctypes.byref(w0))
    scd.lib().scd_sizes(ctypes.byref(sp1), ctypes.byref(a), ctypes.byref(w1))
    assert w1.value >= w0.value + 16 * 16 * 16 * 12 * 8


def test_tile_list():
    rows = scd.tile_list()
    assert len(rows) >= 4 and all(len(r) == 4 for r in rows)
    assert any(r[:2] == (64, 4) for r in rows)
    assert scd.variant_index(*rows[1]) == 1


def test_batch_sizes_reject_mixed_dtypes():
    ps = (B.ScdParams * 2)(B.make_params(W.params(16, 16, 16, 0.1)),
                           B.make_params(W.params(16, 16, 16, 0.1, dtype="f32")))
    n = ctypes.c_size_t()
    assert scd.lib().scd_batch_sizes(2, ps, ctypes.byref(n)) == B.SCD_EINVAL


def test_host_angle_formulas_match_oracle():
    """Young's equation and Huang's estimate are host arithmetic in the
    library; they must agree with the oracle's for both pseudopotentials."""
    import oracle as O
    import workloads as W
    for t in ((0.03, 0.03, 0.05), (0.05, 0.02, 0.06), (0.02, 0.05, 0.06), (0.3, 0.0, 0.05)):
        assert scd.binding.young_angle(*t) == pytest.approx(O.young_angle(*t), abs=1e-12)
    for psi in (0, 1):
        for d in (-0.4, -0.1, 0.0, 0.3):
            p = W.params(8, 8, 8, 0.12, rho_wall=W.asymmetric_wall(d), psi=psi)
            assert scd.binding.huang_angle(p, 0.74, 0.01) == pytest.approx(
                O.huang_angle(p, 0.74, 0.01), abs=1e-12)


def test_stream_copy_rejects_bad_arguments():
    """Argument checks return before any device call."""
    lib = scd.lib()
    assert lib.scd_stream_copy(None, None, 8, None) == B.SCD_EINVAL
    assert lib.scd_stream_copy(4096, 8192, 12, None) == B.SCD_EINVAL      # not a multiple of 8
    assert lib.scd_stream_copy(4100, 8192, 16, None) == B.SCD_EINVAL      # misaligned source
    assert lib.scd_stream_copy(4096, 4104, 64, None) == B.SCD_EINVAL      # overlapping


def test_moment_cache_rejects_bad_arguments():
    lib = scd.lib()
    assert lib.scd_ckpt_moment_cache(None, None, 0) == B.SCD_EINVAL
    assert lib.scd_pull_copy(None) == B.SCD_EINVAL
