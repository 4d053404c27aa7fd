"""CPU checks of the C ABI: the library loads, exports every declared symbol,
validates descriptions, and its host-side tables and addressing are right.
No compute call is made here (no GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pflbm.h")


def _lib():
    from paper_2206_11637_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libpflbm.so not built")
    return L, L.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pflbm_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L, lib = _lib()
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares exactly the header's functions
    assert sorted(L.SIGNATURES) == names


def test_workspace_sizes_and_invalid_descriptions():
    L, lib = _lib()
    d = L.Desc(32, 32, 32, 5, 0, 1, 0)
    n64 = lib.pflbm_workspace_bytes(C.byref(d))
    N = 32 ** 3
    assert n64 >= (42 * 8 + 2 * 8) * N
    d32 = L.Desc(32, 32, 32, 5, 1, 1, 0)
    d16 = L.Desc(32, 32, 32, 5, 2, 1, 1)
    assert lib.pflbm_workspace_bytes(C.byref(d32)) >= (2 * 42 * 4 + 8) * N
    assert lib.pflbm_workspace_bytes(C.byref(d16)) >= (2 * 42 * 2 + 8 + 1 + 4) * N
    # the in-place AA scheme keeps one population buffer
    a32 = L.Desc(32, 32, 32, 5, 1, 1, 0, 1)
    assert (42 * 4 + 8) * N <= lib.pflbm_workspace_bytes(C.byref(a32)) < (2 * 42 * 4) * N
    for bad in (L.Desc(0, 4, 4, 0, 0, 0, 0), L.Desc(4, 4, 4, 9, 0, 0, 0),
                L.Desc(4, 4, 4, 0, 3, 0, 0), L.Desc(4, 4, 4, 0, 0, 2, 0),
                L.Desc(4, 4, 4, 0, 0, 0, 0, 2), L.Desc(4, 4, 4, 0, 0, 0, 0, 0, 2),
                L.Desc(4, 4, 4, 0, 0, 0, 0, 0, -1)):
        assert lib.pflbm_workspace_bytes(C.byref(bad)) == 0
    # Guo's full source is a kernel variant: the same workspace
    assert lib.pflbm_workspace_bytes(C.byref(L.Desc(8, 8, 8, 7, 1, 1, 0, 0, 1))) == \
        lib.pflbm_workspace_bytes(C.byref(L.Desc(8, 8, 8, 7, 1, 1, 0, 0, 0)))
    ctx = C.c_void_p()
    assert lib.pflbm_create(C.byref(L.Desc(0, 4, 4, 0, 0, 0, 0)), C.c_void_p(256), 1 << 20,
                            None, C.byref(ctx)) == L.PFLBM_ERR_ARG
    assert lib.pflbm_create(C.byref(d), C.c_void_p(256), 10, None, C.byref(ctx)) == L.PFLBM_ERR_ARG
    assert lib.pflbm_status_string(L.PFLBM_ERR_UNSTABLE).decode().startswith("unstable")


@pytest.mark.parametrize("precision,nz_ok", [(0, 511), (1, 1023), (2, 1023)])
def test_lattice_size_limits_are_checked_on_the_host(precision, nz_ok):
    """The largest accepted lattice of a 1024 x 512 cross-section (2 N times the
    value size below 2^32), one plane more is refused; products that overflow
    64 bits and thin shapes whose launch grid reaches 2^32 work-items are
    refused too."""
    L, lib = _lib()
    def ws(nx, ny, nz):
        return lib.pflbm_workspace_bytes(C.byref(L.Desc(nx, ny, nz, 0, precision, 1, 0)))
    assert ws(1024, 512, nz_ok) > 0
    assert ws(1024, 512, nz_ok + 1) == 0
    for dims in ((1 << 21,) * 3, (2 ** 31 - 1,) * 3, (1 << 30, 1 << 30, 4), (1, 1 << 30, 1 << 30)):
        assert ws(*dims) == 0, dims
    # 1 x 1 x nz: one 16 x 16 tile per plane, 256 work-items per cell
    assert ws(1, 1, (1 << 24) - 1) > 0
    assert ws(1, 1, 1 << 24) == 0


def test_parameter_validation_without_a_gpu():
    """set_params checks arguments on the host (the workspace pointer is never
    dereferenced by create/set_params/destroy)."""
    L, lib = _lib()
    d = L.Desc(8, 8, 8, 7, 1, 1, 0)
    n = lib.pflbm_workspace_bytes(C.byref(d))
    ctx = C.c_void_p()
    assert lib.pflbm_create(C.byref(d), C.c_void_p(4096), n, None, C.byref(ctx)) == 0
    import workloads as W
    from paper_2206_11637_amd.sim import _params_struct
    good = _params_struct(W.Params())
    assert lib.pflbm_set_params(ctx, C.byref(good)) == 0
    for field, val in (("tau_H", 0.5), ("mobility", 0.0), ("xi", -1.0), ("sigma", -1e-4),
                       ("rho_L", 0.0), ("s_high", 2.0), ("s_bulk", 2.0), ("s_bulk", -0.5),
                       ("rho_g_ref", float("inf")), ("rho_g_ref", float("nan"))):
        p = _params_struct(W.Params())
        setattr(p, field, val)
        assert lib.pflbm_set_params(ctx, C.byref(p)) == L.PFLBM_ERR_ARG, field
        assert len(lib.pflbm_last_error(ctx)) > 0
    for sb in (0.0, 1.0, 1.99):
        p = _params_struct(W.Params(s_bulk=sb))
        assert lib.pflbm_set_params(ctx, C.byref(p)) == 0, sb
    for ref in (0.0, 1.0, -0.5):
        p = _params_struct(W.Params(rho_g_ref=ref))
        assert p.rho_g_ref == ref
        assert lib.pflbm_set_params(ctx, C.byref(p)) == 0, ref
    p = _params_struct(W.Params())
    p.fp16_scale_log2[0] = 3.5
    assert lib.pflbm_set_params(ctx, C.byref(p)) == L.PFLBM_ERR_ARG
    # stepping before init is a state error, not a crash
    assert lib.pflbm_step(ctx, 1) == L.PFLBM_ERR_STATE
    # saved-state steps: bad buffers and unknown flags are rejected on the host
    a, b = C.c_void_p(1 << 20), C.c_void_p(1 << 21)
    assert lib.pflbm_step_states(ctx, a, a, 0, 0) == L.PFLBM_ERR_ARG
    assert lib.pflbm_step_states(ctx, a, b, -1, 0) == L.PFLBM_ERR_ARG
    assert lib.pflbm_step_states(ctx, a, b, 0, 4) == L.PFLBM_ERR_ARG
    assert lib.pflbm_set_check_interval(ctx, -1) == L.PFLBM_ERR_ARG
    assert lib.pflbm_destroy(ctx) == 0
    # the chained-recompute flags need the two-buffer scheme
    daa = L.Desc(8, 8, 8, 7, 1, 1, 0, L.STREAMING["aa"])
    n = lib.pflbm_workspace_bytes(C.byref(daa))
    ctx = C.c_void_p()
    assert lib.pflbm_create(C.byref(daa), C.c_void_p(4096), n, None, C.byref(ctx)) == 0
    assert lib.pflbm_step_states(ctx, a, b, 0, L.STATES_WRITE_SRC_PHI) == L.PFLBM_ERR_ARG
    assert "PFLBM_STREAM_AB" in lib.pflbm_last_error(ctx).decode()
    assert lib.pflbm_destroy(ctx) == 0


def test_d3q27_phase_build_loads_and_exports_every_symbol():
    """The D3Q27-phase build is the same interface: every declared symbol,
    pflbm_phase_q() = 27 (and 15 for the default build), its velocity set the
    oracle's D3Q27, and 15 rejected as a lattice size."""
    from oracle import lattice as OL
    from paper_2206_11637_amd import _lib as L
    from paper_2206_11637_amd.sim import lattice
    if not os.path.exists(L.LIB_PATHS["d3q27"]):
        pytest.skip("libpflbm_d3q27.so not built")
    lib27 = L.load(phase="d3q27")
    for name in declared_functions():
        assert hasattr(lib27, name), name
    assert lib27.pflbm_phase_q() == 27
    assert L.load().pflbm_phase_q() == 15
    c, w = lattice(27, "d3q27")
    assert sorted(map(tuple, c)) == sorted(map(tuple, OL.D3Q27.c_np))
    assert lib27.pflbm_lattice(15, None, None) == L.PFLBM_ERR_ARG
    # 27 h per cell: the workspace grows by 12 populations per cell and buffer
    d = L.Desc(8, 8, 8, 7, 1, 1, 0)
    n15, n27 = L.load().pflbm_workspace_bytes(C.byref(d)), lib27.pflbm_workspace_bytes(C.byref(d))
    assert n27 - n15 >= 2 * 12 * 4 * 512


def test_library_velocity_sets_match_the_oracle_lattices():
    from oracle import lattice as OL
    from paper_2206_11637_amd.sim import lattice
    for q, lat in ((15, OL.D3Q15), (27, OL.D3Q27)):
        c, w = lattice(q)
        assert sorted(map(tuple, c)) == sorted(map(tuple, lat.c_np))
        wo = {tuple(v): lat.w_np[i] for i, v in enumerate(lat.c_np)}
        for i in range(q):
            assert abs(w[i] - wo[tuple(c[i])]) < 1e-16
        # opposite pairs are adjacent (the kernels rely on it)
        for i in range(1, q, 2):
            assert (c[i] == -c[i + 1]).all()


def xcd_remap(b, nb):
    """Host restatement of the kernels' block renumbering (checked to be a bijection)."""
    q, r, x, k = nb >> 3, nb & 7, b & 7, b >> 3
    return x * (q + 1) + k if x < r else r * (q + 1) + (x - r) * q + k


@pytest.mark.parametrize("nb", [1, 7, 8, 9, 64, 1001, 65536 + 5])
def test_xcd_remap_is_a_bijection_with_contiguous_ranges(nb):
    b = np.arange(nb)
    out = np.array([xcd_remap(int(v), nb) for v in b])
    assert sorted(out.tolist()) == list(range(nb))
    for x in range(8):
        sel = np.sort(out[b % 8 == x])
        if len(sel):
            assert (np.diff(sel) == 1).all()


def _pull_map(nx, ny, nz, periodic, solid, c):
    """Slot (population, cell) each fluid cell pulls population i from, under
    the two-buffer pull rule the kernels use: slot(i, y - c_i) if y - c_i is
    fluid, else the bounce-back slot(opp i, y)."""
    q = len(c)
    opp = [0] + [i + 1 if i % 2 else i - 1 for i in range(1, q)]

    def nb(x, y, z, d):
        X, Y, Z = x + d[0], y + d[1], z + d[2]
        for v, n, p in ((X, nx, periodic[0]), (Y, ny, periodic[1]), (Z, nz, periodic[2])):
            if (v < 0 or v >= n) and not p:
                return None
        X, Y, Z = X % nx, Y % ny, Z % nz
        idx = X + nx * (Y + ny * Z)
        return None if solid[idx] else idx

    reads = {}
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                idx = x + nx * (y + ny * z)
                if solid[idx]:
                    continue
                for i in range(q):
                    s = nb(x, y, z, -c[i]) if i else idx
                    reads[(i, idx)] = (opp[i], idx) if s is None else (i, s)
    return reads, opp


@pytest.mark.parametrize("q", [15, 27])
def test_pull_streaming_reads_each_slot_once_and_is_streaming(q):
    """The pull rule reads every fluid slot of the previous state exactly once
    (a permutation), and what cell y receives in direction i is what cell
    y - c_i emitted in direction i, or its own emission in direction opp i
    behind a wall or solid (halfway bounce-back)."""
    from oracle import lattice as OL
    c = (OL.D3Q15 if q == 15 else OL.D3Q27).c_np
    # the library's order: rest, then opposite pairs adjacent
    order = [0]
    used = {0}
    for i in range(1, q):
        if i in used:
            continue
        j = [k for k in range(q) if (c[k] == -c[i]).all()][0]
        order += [i, j]
        used |= {i, j}
    c = c[order]
    rng = np.random.default_rng(0)
    nx, ny, nz = 5, 4, 3
    solid = rng.uniform(size=nx * ny * nz) < 0.15
    fluid_slots = {(i, idx) for i in range(q) for idx in range(nx * ny * nz) if not solid[idx]}
    for periodic in ((True, False, True), (False, False, False), (True, True, True)):
        reads, opp = _pull_map(nx, ny, nz, periodic, solid, c)
        src = list(reads.values())
        assert len(set(src)) == len(src) == len(fluid_slots) and set(src) == fluid_slots
        for (i, y), (j, x) in reads.items():
            if j == i and x != y:
                X = np.array([x % nx, (x // nx) % ny, x // (nx * ny)])
                Y = np.array([y % nx, (y // nx) % ny, y // (nx * ny)])
                d = (Y - X - c[i] + np.array([nx, ny, nz])) % np.array([nx, ny, nz])
                assert (d == 0).all()
            elif i:
                assert j == opp[i] and x == y


def _aa_maps(nx, ny, nz, periodic, solid, c, odd):
    """Slots (population, cell) read and written by each fluid cell under the
    in-place AA rules, as the kernels compute them."""
    q = len(c)
    opp = [0] + [i + 1 if i % 2 else i - 1 for i in range(1, q)]
    N = nx * ny * nz

    def nb(x, y, z, d):
        X, Y, Z = x + d[0], y + d[1], z + d[2]
        for v, n, p in ((X, nx, periodic[0]), (Y, ny, periodic[1]), (Z, nz, periodic[2])):
            if (v < 0 or v >= n) and not p:
                return None
        X, Y, Z = X % nx, Y % ny, Z % nz
        idx = X + nx * (Y + ny * Z)
        return None if solid[idx] else idx

    reads, writes = [], []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                idx = x + nx * (y + ny * z)
                if solid[idx]:
                    continue
                for i in range(q):
                    if not odd:
                        reads.append((i, idx))
                        writes.append((opp[i], idx))
                    else:
                        s = nb(x, y, z, -c[i])
                        reads.append((i, idx) if s is None else (opp[i], s))
                        d = nb(x, y, z, c[i])
                        writes.append((opp[i], idx) if d is None else (i, d))
    return reads, writes


@pytest.mark.parametrize("q", [15, 27])
def test_aa_pattern_reads_and_writes_each_slot_once(q):
    """Race freedom of the in-place streaming: per parity, the read slots and
    the written slots are each a permutation of the fluid slots, and the odd
    step writes exactly the slots the next even step reads (and vice versa)."""
    from oracle import lattice as OL
    c = (OL.D3Q15 if q == 15 else OL.D3Q27).c_np
    # use the library's order (pairs adjacent) via sorting into pairs
    order = [0]
    used = {0}
    for i in range(1, q):
        if i in used:
            continue
        j = [k for k in range(q) if (c[k] == -c[i]).all()][0]
        order += [i, j]
        used |= {i, j}
    c = c[order]
    rng = np.random.default_rng(0)
    nx, ny, nz = 5, 4, 3
    solid = rng.uniform(size=nx * ny * nz) < 0.15
    fluid_slots = {(i, idx) for i in range(q) for idx in range(nx * ny * nz) if not solid[idx]}
    for periodic in ((True, False, True), (False, False, False), (True, True, True)):
        for odd in (False, True):
            r, w = _aa_maps(nx, ny, nz, periodic, solid, c, odd)
            assert len(set(r)) == len(r) == len(fluid_slots) and set(r) == fluid_slots
            assert len(set(w)) == len(w) == len(fluid_slots) and set(w) == fluid_slots


def test_static_reduction_refuses_lattices_beyond_its_scratch():
    """pflbm_reduce_static rejects, on the host and before touching the GPU, a
    lattice whose partial sums exceed the 16 MiB static array (1024 x 1024 x
    256 cells: 4096 tiles x 256 planes x 40 bytes), and names the sizes."""
    L, lib = _lib()
    d = L.Desc(1024, 1024, 256, 7, 1, 1, 0)
    n = lib.pflbm_workspace_bytes(C.byref(d))
    assert n > 0
    ctx = C.c_void_p()
    assert lib.pflbm_create(C.byref(d), C.c_void_p(4096), n, None, C.byref(ctx)) == 0
    out = (C.c_double * 5)()
    assert lib.pflbm_reduce_static(ctx, out) == L.PFLBM_ERR_ARG
    msg = lib.pflbm_last_error(ctx).decode()
    assert "static scratch" in msg and str(16 << 20) in msg
    assert lib.pflbm_reduce_static(ctx, None) == L.PFLBM_ERR_ARG
    assert lib.pflbm_destroy(ctx) == 0
    # a lattice within the limit gets past the size check to the state check
    d = L.Desc(384, 384, 384, 5, 1, 1, 0)
    n = lib.pflbm_workspace_bytes(C.byref(d))
    assert lib.pflbm_create(C.byref(d), C.c_void_p(4096), n, None, C.byref(ctx)) == 0
    assert lib.pflbm_reduce_static(ctx, out) == L.PFLBM_ERR_STATE
    assert lib.pflbm_destroy(ctx) == 0


def test_binding_refuses_mismatched_buffers_on_the_host():
    """The binding's buffer checks (run before any library call): wrong
    length, dtype, device, contiguity or size raise ValueError; matching
    buffers pass.  CPU tensors stand in for device buffers here."""
    import torch

    from paper_2206_11637_amd.sim import check_buffer
    cpu = torch.device("cpu")
    ok = torch.zeros(10, dtype=torch.float64)
    assert check_buffer(ok, cpu, "x", numel=10, dtype=torch.float64) is ok
    bad = [
        (torch.zeros(9, dtype=torch.float64), dict(numel=10, dtype=torch.float64), "values"),
        (torch.zeros(10, dtype=torch.float32), dict(numel=10, dtype=torch.float64), "dtype"),
        (torch.zeros(20, dtype=torch.float64)[::2], dict(numel=10), "contiguous"),
        (torch.zeros(100, dtype=torch.uint8), dict(min_bytes=101), "bytes"),
        (ok.numpy(), dict(numel=10), "tensor"),
    ]
    for t, kw, word in bad:
        with pytest.raises(ValueError, match=word):
            check_buffer(t, cpu, "x", **kw)
    with pytest.raises(ValueError, match="simulation is on"):
        check_buffer(ok, torch.device("cuda:0"), "x")


def test_copy_probe_refuses_bad_arguments_before_any_launch():
    """pflbm_hbm_copy checks pointers, alignment, size and form on the host
    and enqueues nothing when one is wrong (stand-in addresses, never
    dereferenced)."""
    L, lib = _lib()
    src, dst = C.c_void_p(1 << 20), C.c_void_p(1 << 21)
    soa = 43 * 4 * 256
    err = L.PFLBM_ERR_ARG
    assert lib.pflbm_hbm_copy(None, dst, 1024, L.COPY_FORMS["w4"], None) == err
    assert lib.pflbm_hbm_copy(src, src, 1024, L.COPY_FORMS["w4"], None) == err
    assert lib.pflbm_hbm_copy(src, dst, 0, L.COPY_FORMS["w4"], None) == err
    assert lib.pflbm_hbm_copy(C.c_void_p((1 << 20) + 4), dst, 1024, L.COPY_FORMS["w16"], None) == err
    assert lib.pflbm_hbm_copy(src, dst, 1000, L.COPY_FORMS["w16"], None) == err
    for form in ("soa43", "soa43_nt", "soa43_f64", "soa43_f64_nt"):
        assert lib.pflbm_hbm_copy(src, dst, soa + 16, L.COPY_FORMS[form], None) == err
    assert lib.pflbm_hbm_copy(src, dst, 1024, max(L.COPY_FORMS.values()) + 1, None) == err
    assert lib.pflbm_hbm_copy(src, dst, 1024, -1, None) == err


@pytest.mark.parametrize("precision, size", [(0, 8), (1, 4), (2, 2)])
def test_face_pack_size_and_refusals_on_the_host(precision, size):
    """pflbm_pack_faces reports 2 faces x (5 h + 9 g rows with c_z = -/+1) x
    nx x ny values of the storage size and refuses, before any launch, a
    missing size pointer, a short buffer, the in-place scheme and a state that
    was never initialised (stand-in addresses, never dereferenced)."""
    L, lib = _lib()
    from paper_2206_11637_amd.sim import lattice
    c_h, c_g = lattice(int(lib.pflbm_phase_q()))[0], lattice(27)[0]
    rows = int((c_h[:, 2] == 1).sum() + (c_g[:, 2] == 1).sum())
    assert rows == ((9 if lib.pflbm_phase_q() == 27 else 5) + 9)
    d = L.Desc(12, 7, 5, 7, precision, 1, 0)
    n = lib.pflbm_workspace_bytes(C.byref(d))
    ctx = C.c_void_p()
    assert lib.pflbm_create(C.byref(d), C.c_void_p(4096), n, None, C.byref(ctx)) == 0
    need = C.c_size_t()
    assert lib.pflbm_pack_faces(None, None, 0, C.byref(need)) == L.PFLBM_ERR_ARG
    assert lib.pflbm_pack_faces(ctx, None, 0, None) == L.PFLBM_ERR_ARG
    assert lib.pflbm_pack_faces(ctx, None, 0, C.byref(need)) == 0
    assert need.value == 2 * rows * 12 * 7 * size
    dst = C.c_void_p(1 << 20)
    assert lib.pflbm_pack_faces(ctx, dst, need.value - 1, C.byref(need)) == L.PFLBM_ERR_ARG
    if size > 1:
        assert lib.pflbm_pack_faces(ctx, C.c_void_p((1 << 20) + 1), need.value,
                                    C.byref(need)) == L.PFLBM_ERR_ARG
    assert lib.pflbm_pack_faces(ctx, dst, need.value, C.byref(need)) == L.PFLBM_ERR_STATE
    assert lib.pflbm_destroy(ctx) == 0
    daa = L.Desc(12, 7, 5, 7, precision, 1, 0, L.STREAMING["aa"])
    n = lib.pflbm_workspace_bytes(C.byref(daa))
    assert lib.pflbm_create(C.byref(daa), C.c_void_p(4096), n, None, C.byref(ctx)) == 0
    assert lib.pflbm_pack_faces(ctx, dst, need.value, C.byref(need)) == L.PFLBM_ERR_STATE
    assert "PFLBM_STREAM_AB" in lib.pflbm_last_error(ctx).decode()
    assert lib.pflbm_destroy(ctx) == 0
