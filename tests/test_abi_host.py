"""Host-side checks of libsph that need no GPU: the library loads, exports
every symbol include/sph.h declares, the ctypes structs match the C layout,
and argument validation rejects bad calls before any device work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def S():
    from paper_2104_00537_amd import sph
    return sph


def test_library_exports_every_declared_symbol(S):
    decl = _declared()
    assert decl == sorted(S.EXPORTS)
    lib = C.CDLL(S.LIB_PATH)
    for name in decl:
        assert hasattr(lib, name), name


def test_struct_layout_matches_header(S, tmp_path):
    """The ctypes mirrors have the C compiler's size and field offsets."""
    fields = [f for f, _ in S.SphParams._fields_]
    sfields = [f for f, _ in S.SphState._fields_]
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "sph.h"', "int main(void){",
            'printf("%zu %zu\\n", sizeof(sph_params), sizeof(sph_state));']
    prog += [f'printf("%zu\\n", offsetof(sph_params, {f}));' for f in fields]
    prog += [f'printf("%zu\\n", offsetof(sph_state, {f}));' for f in sfields]
    prog += ["return 0;}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(prog))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == C.sizeof(S.SphParams) and vals[1] == C.sizeof(S.SphState)
    assert vals[2:2 + len(fields)] == [getattr(S.SphParams, f).offset for f in fields]
    assert vals[2 + len(fields):] == [getattr(S.SphState, f).offset for f in sfields]


def test_body_layout_matches_header(S, tmp_path):
    """The ctypes mirror of sph_body has the C size and field offsets."""
    fields = [f for f, _ in S.SphBody._fields_]
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "sph.h"', "int main(void){",
            'printf("%zu %d\\n", sizeof(sph_body), SPH_MAX_BODIES);']
    prog += [f'printf("%zu\\n", offsetof(sph_body, {f}));' for f in fields]
    prog += ["return 0;}"]
    src = tmp_path / "body.c"
    src.write_text("\n".join(prog))
    exe = tmp_path / "body"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    vals = [int(v) for v in
            subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert vals[0] == C.sizeof(S.SphBody) and vals[1] == S.SPH_MAX_BODIES
    assert vals[2:] == [getattr(S.SphBody, f).offset for f in fields]


def test_floating_step_validates_without_device(S):
    """sph_floating_step rejects a case without floating = 1, a body count
    outside [1, SPH_MAX_BODIES], a missing table or particle ids, and a bad
    phase; floating bodies cannot be combined with modified DBC, the
    precision-study arms or the batched path."""
    from paper_2104_00537_amd import cases
    c = cases.floating_box(2, dp=0.04)
    P = S.make_params(c.params)
    assert P.floating == 1
    lib = S.lib
    d = C.c_void_p(16)
    st = S.SphState(16, 16, 16, 16, 16, None)
    noid = S.SphState(16, 16, 16, 16, None, None)
    need = S.sph_workspace_bytes(P, 1000)

    def call(p=P, phase=0, bodies=d, nb=1, s=st, ws=need):
        return lib.sph_floating_step(C.byref(p), 1000, phase, d, bodies, nb, C.byref(st),
                                     C.byref(s), d, d, ws, None)

    assert call(nb=0) == S.SPH_E_ARG
    assert call(nb=S.SPH_MAX_BODIES + 1) == S.SPH_E_ARG
    assert call(bodies=None) == S.SPH_E_ARG
    assert call(s=noid) == S.SPH_E_ARG
    assert call(phase=2) == S.SPH_E_ARG
    assert call(ws=need - 1) == S.SPH_E_WORKSPACE
    P0 = S.make_params(c.params)
    P0.floating = 0
    assert call(p=P0) == S.SPH_E_ARG
    P1 = S.make_params(c.params)
    P1.boundary = 1
    assert call(p=P1) == S.SPH_E_ARG
    # the precision-study arms take the default formulation only, with or
    # without the one-lane flag
    for flags in (S.SPH_INTERACT_F64, S.SPH_INTERACT_ABS_F32,
                  S.SPH_INTERACT_F64 | S.SPH_INTERACT_ONE_LANE,
                  S.SPH_INTERACT_ABS_F32 | S.SPH_INTERACT_ONE_LANE):
        assert lib.sph_interact(C.byref(P), 1000, C.byref(st), d, d, d, d, None, None, flags, d,
                                need, None) == S.SPH_E_ARG
    with pytest.raises(S.SphError):
        S.sph_batch_describe([S.make_params(cases.dam_break_2d(dp=0.05).params), P],
                             [0, 10, 20])


def test_workspace_bytes_monotone(S):
    from paper_2104_00537_amd import cases
    P = S.make_params(cases.dam_break_2d().params)
    sizes = [S.sph_workspace_bytes(P, n) for n in (0, 1, 1000, 100000, 10 ** 7)]
    assert all(a <= b for a, b in zip(sizes, sizes[1:]))
    assert sizes[-1] > 10 ** 7 * 48
    assert S.sph_workspace_bytes(P, -1) == 0


def _bad_params(S, **kw):
    from paper_2104_00537_amd import cases
    P = S.make_params(cases.dam_break_2d().params)
    for k, v in kw.items():
        if k == "ncell":
            for i, x in enumerate(v):
                P.ncell[i] = x
        else:
            setattr(P, k, v)
    return P


@pytest.mark.parametrize("kw", [
    dict(dim=4), dict(dim=1), dict(cell_div=3), dict(h=0.0), dict(c0=-1.0),
    dict(ncell=(0, 5, 1)), dict(ncell=(5, 5, 2)), dict(cell_size=0.001),
    dict(ncell=(70000, 70000, 1)), dict(mass_fluid=0.0), dict(gamma=0.0),
])
def test_argument_validation_without_device(S, kw):
    """Bad parameters are rejected with SPH_E_ARG before any HIP call."""
    P = _bad_params(S, **kw)
    dummy = C.c_void_p(16)
    st = S.SphState(16, 16, 16, 16, None)
    lib = S.lib
    r = lib.sph_bin_cells(C.byref(P), 10, C.byref(st), C.byref(st), None, None, dummy, dummy,
                          dummy, dummy, 1 << 30, None)
    assert r == S.SPH_E_ARG
    r = lib.sph_interact(C.byref(P), 10, C.byref(st), dummy, dummy, dummy, dummy, None, None, 0,
                         dummy, 1 << 30, None)
    assert r == S.SPH_E_ARG
    r = lib.sph_reduce_dt(C.byref(P), 10, dummy, None, None, dummy, 1 << 30, None)
    assert r == S.SPH_E_ARG
    r = lib.sph_symplectic_step(C.byref(P), 10, 0, dummy, dummy, C.byref(st), C.byref(st), dummy,
                                dummy, dummy, 1 << 30, None)
    assert r == S.SPH_E_ARG


def test_workspace_and_pointer_checks_without_device(S):
    from paper_2104_00537_amd import cases
    P = S.make_params(cases.dam_break_2d().params)
    lib = S.lib
    d = C.c_void_p(16)
    st = S.SphState(16, 16, 16, 16, None)
    st2 = S.SphState(32, 16, 16, 16, None)
    need = S.sph_workspace_bytes(P, 1000)
    assert lib.sph_bin_cells(C.byref(P), 1000, C.byref(st), C.byref(st2), None, None, d, d, d, d,
                             need - 1, None) == S.SPH_E_WORKSPACE
    # in and out aliasing
    assert lib.sph_bin_cells(C.byref(P), 1000, C.byref(st), C.byref(st), None, None, d, d, d, d,
                             need, None) == S.SPH_E_ARG
    # only one side of the carry pair
    assert lib.sph_bin_cells(C.byref(P), 1000, C.byref(st), C.byref(st2), C.byref(st), None, d, d,
                             d, d, need, None) == S.SPH_E_ARG
    # null outputs
    assert lib.sph_interact(C.byref(P), 1000, C.byref(st), d, d, None, d, None, None, 0, d, need,
                            None) == S.SPH_E_ARG
    # an unknown flag bit (0x20), and unknown bits with the known ones
    for fl in (0x20, 0x20 | S.SPH_INTERACT_ONE_LANE, 0x40 | S.SPH_DIAG_COUNT_F64):
        assert lib.sph_interact(C.byref(P), 1000, C.byref(st), d, d, d, d, None, None, fl, d,
                                need, None) == S.SPH_E_ARG
    assert lib.sph_symplectic_step(C.byref(P), 1000, 2, d, d, C.byref(st), C.byref(st), d, d, d,
                                   need, None) == S.SPH_E_ARG
    assert lib.sph_read_error(None) == S.SPH_E_ARG
    assert lib.sph_strerror(S.SPH_E_WORKSPACE) == b"workspace too small"


def test_noalloc_validates_without_device(S):
    """sph_interact_noalloc rejects sizes beyond its array, modified DBC,
    reused cells and bad parameters before any HIP call."""
    from paper_2104_00537_amd import cases
    P = S.make_params(cases.dam_break_2d().params)
    lib = S.lib
    d = C.c_void_p(16)
    st = S.SphState(16, 16, 16, 16, None)
    call = lambda P, n, fl=0: lib.sph_interact_noalloc(C.byref(P), n, C.byref(st), d, d, d, d,
                                                       None, None, fl, None)
    assert call(P, S.SPH_NOALLOC_MAX_N + 1) == S.SPH_E_ARG
    assert call(P, -1) == S.SPH_E_ARG
    assert call(P, 1000, S.SPH_INTERACT_REUSE_CELLS) == S.SPH_E_ARG
    assert call(P, 1000, 0x20) == S.SPH_E_ARG
    assert call(_bad_params(S, h=0.0), 1000) == S.SPH_E_ARG
    assert call(_bad_params(S, boundary=1), 1000) == S.SPH_E_ARG
    assert lib.sph_interact_noalloc(C.byref(P), 1000, C.byref(st), d, d, None, d, None, None, 0,
                                    None) == S.SPH_E_ARG


def test_list_calls_validate_without_device(S):
    """The neighbour-list calls reject what they do not take (formulation
    options, FP64 state, bad skin or flags, short buffers) before any HIP
    call, and size the buffer as header + counts + 40 chunks per target."""
    from paper_2104_00537_amd import cases
    c = cases.dam_break_2d()
    P = S.make_params(c.params)
    lib = S.lib
    n = 1000
    assert S.sph_list_bytes(P, n) == 256 + (4 * n + 255) // 256 * 256 + 8 * n * 40
    for kw in (dict(kernel=1), dict(viscosity=1), dict(ddt=2), dict(boundary=1),
               dict(floating=1), dict(h=0.0)):
        assert S.sph_list_bytes(_bad_params(S, **kw), n) == 0, kw
    assert S.sph_list_bytes(P, -1) == 0
    d = C.c_void_p(16)
    st = S.SphState(16, 16, 16, 16, None)
    st64 = S.SphState(16, 16, 16, 16, None, None, 16, 16)
    lb = S.sph_list_bytes(P, n)
    ws = S.sph_workspace_bytes(P, n)
    cs = float(c.params.cell_size)

    def build(skin=0.0, fl=0, lbytes=lb, wbytes=ws, state=st, lst=d):
        return lib.sph_build_list(C.byref(P), n, C.byref(state), d, d, skin, fl, lst, lbytes, d,
                                  wbytes, None)

    assert build(fl=2) == S.SPH_E_ARG
    assert build(skin=-1e-9) == S.SPH_E_ARG
    assert build(skin=0.5 * cs) == S.SPH_E_ARG
    assert build(skin=float("nan")) == S.SPH_E_ARG
    assert build(lbytes=lb - 8 * n * 40) == S.SPH_E_ARG  # no room for one chunk per target
    assert build(lst=None) == S.SPH_E_ARG
    assert build(state=st64) == S.SPH_E_ARG
    assert build(wbytes=ws - 1) == S.SPH_E_WORKSPACE

    def replay(fl=0, lbytes=lb, wbytes=ws, state=st, ace=d):
        return lib.sph_interact_list(C.byref(P), n, C.byref(state), d, d, d, lbytes, ace, d, None,
                                     None, fl, d, wbytes, None)

    assert replay(fl=0x20) == S.SPH_E_ARG
    assert replay(lbytes=lb - 8 * n * 40) == S.SPH_E_ARG
    assert replay(ace=None) == S.SPH_E_ARG
    assert replay(state=st64) == S.SPH_E_ARG
    assert replay(wbytes=ws - 1) == S.SPH_E_WORKSPACE
    assert lib.sph_list_walks(None) == S.SPH_E_ARG


def test_batch_describe_host_only(S):
    """The slot table is built on the host: key ranges are the cells of the
    slots before plus one each, offsets are validated, cell_div must agree."""
    from paper_2104_00537_amd import cases
    cs = [cases.dam_break_2d(dp=0.02), cases.block_case(3, (5, 4, 3)),
          cases.dam_break_2d(dp=0.04)]
    P = [S.make_params(c.params) for c in cs]
    offs = [0]
    for c in cs:
        offs.append(offs[-1] + c.n)
    b, host = S.sph_batch_describe(P, offs)
    assert b.n_slots == 3 and b.n_total == offs[-1] and b.cell_div == 1
    assert b.key_cells == sum(c.params.ncell_total() + 1 for c in cs)
    assert host.size == S.lib.sph_batch_table_bytes(3) > 0
    assert S.sph_batch_workspace_bytes(b) >= S.sph_workspace_bytes(P[0], offs[-1])
    with pytest.raises(S.SphError):
        S.sph_batch_describe(P, [1] + offs[1:])            # offsets[0] != 0
    with pytest.raises(S.SphError):
        S.sph_batch_describe(P, [0, offs[2], offs[1], offs[3]])   # decreasing
    cd2 = cases.dam_break_2d(dp=0.02, cell_div=2)
    with pytest.raises(S.SphError):
        S.sph_batch_describe([P[0], S.make_params(cd2.params)], [0, 10, 20])
    assert S.lib.sph_batch_table_bytes(0) == 0
    assert S.lib.sph_batch_table_bytes(S.SPH_BATCH_MAX_SLOTS + 1) == 0


def test_batch_calls_validate_without_device(S):
    lib = S.lib
    b = S.SphBatch(2, 1, 100, 50, None)   # no table: rejected
    d = C.c_void_p(16)
    st = S.SphState(16, 16, 16, 16, None)
    st2 = S.SphState(32, 16, 16, 16, None)
    assert lib.sph_batch_bin_cells(C.byref(b), C.byref(st), C.byref(st2), None, None, d, d, d, d,
                                   1 << 30, None) == S.SPH_E_ARG
    b.table = 16
    assert lib.sph_batch_bin_cells(C.byref(b), C.byref(st), C.byref(st2), None, None, d, d, d, d,
                                   16, None) == S.SPH_E_WORKSPACE
    b.n_total = 1 << 27                    # beyond the packed-index range
    assert lib.sph_batch_interact(C.byref(b), C.byref(st), d, d, d, d, None, None, 0, d, 1 << 40,
                                  None) == S.SPH_E_ARG
    b.n_total = 100
    # flags other than reusing the cells, a workspace too small for a refresh
    for fl in (S.SPH_DIAG_COUNT_F64, S.SPH_INTERACT_F64, 1 << 7):
        assert lib.sph_batch_interact(C.byref(b), C.byref(st), d, d, d, d, None, None, fl, d,
                                      1 << 40, None) == S.SPH_E_ARG
    assert lib.sph_batch_interact(C.byref(b), C.byref(st), d, d, d, d, None, None,
                                  S.SPH_INTERACT_REUSE_CELLS, d, 16, None) == S.SPH_E_WORKSPACE
    assert lib.sph_batch_refresh_view(C.byref(b), C.byref(st), d, d, 16, None) == S.SPH_E_WORKSPACE
    assert lib.sph_batch_refresh_view(C.byref(b), C.byref(st), None, d, 1 << 40,
                                      None) == S.SPH_E_ARG
    assert lib.sph_batch_symplectic_step(C.byref(b), 3, d, d, C.byref(st), C.byref(st), d, d, d,
                                         1 << 30, None) == S.SPH_E_ARG
    # shifting: flags other than reusing the cells, missing dt, FP64 state, small workspace
    st64 = S.SphState(16, 16, 16, 16, None, None, 16, 16)
    shift = lambda fl=0, dt=d, state=st, wb=1 << 40: lib.sph_batch_shifting(  # noqa: E731
        C.byref(b), C.byref(state), d, d, dt, None, None, fl, d, wb, None)
    assert shift(fl=S.SPH_DIAG_COUNT_F64) == S.SPH_E_ARG
    assert shift(dt=None) == S.SPH_E_ARG
    assert shift(state=st64) == S.SPH_E_ARG
    assert shift(fl=S.SPH_INTERACT_REUSE_CELLS, wb=16) == S.SPH_E_WORKSPACE


def test_batch_describe_sets_the_wave_alignment_flag(S):
    """SPH_BATCH_WAVE_ALIGNED iff every slot offset is a multiple of 64."""
    from paper_2104_00537_amd import cases
    P = S.make_params(cases.dam_break_2d(dp=0.02).params)
    for offs, want in (([0, 64, 192], True), ([0, 64, 190], False), ([0, 60, 128], False),
                       ([0, 0, 128], True)):
        b, _ = S.sph_batch_describe([P, P], offs)
        assert bool(b.flags & S.SPH_BATCH_WAVE_ALIGNED) == want, offs


def test_batch_describe_lanes_per_slot(S):
    """One lane per target unless SPH_BATCH_FOUR_LANES is asked for; then, in
    a wave-aligned batch, four for each slot of at most 131,072 particles
    (by its own size), one for larger slots."""
    import ctypes as C
    from paper_2104_00537_amd import cases
    P = S.make_params(cases.dam_break_2d(dp=0.02).params)
    small, big = 64 * 100, 64 * 2100  # 6,400 and 134,400 particles
    offs = [0, small, small + big, 2 * small + big]
    b, _ = S.sph_batch_describe([P, P, P], offs)
    assert b.lanes == offs[-1] and not b.flags & S.SPH_BATCH_FOUR_LANES
    b, _ = S.sph_batch_describe([P, P, P], offs, four_lanes=True)
    assert b.flags & S.SPH_BATCH_FOUR_LANES and b.flags & S.SPH_BATCH_WAVE_ALIGNED
    assert b.lanes == 4 * small + big + 4 * small
    b, _ = S.sph_batch_describe([P, P], [0, 100, 228], four_lanes=True)  # not aligned
    assert b.lanes == 228 and not b.flags & (S.SPH_BATCH_FOUR_LANES | S.SPH_BATCH_WAVE_ALIGNED)
    ps = (S.SphParams * 1)(P)
    o = (C.c_int64 * 2)(0, 64)
    host = (C.c_uint8 * S.lib.sph_batch_table_bytes(1))()
    bb = S.SphBatch()
    assert S.lib.sph_batch_describe(ps, o, 1, 4, host, C.sizeof(host), C.byref(bb)) == S.SPH_E_ARG
    assert S.lib.sph_batch_describe(ps, o, 1, 2, host, C.sizeof(host), C.byref(bb)) == S.SPH_OK


def test_batch_describe_formulation_options(S):
    """Slots may take formulation options (cubic spline, laminar viscosity,
    Fourtakas DDT; SPH_BATCH_GENERAL iff some slot does) and periodic
    components (SPH_BATCH_PERIODIC); modified DBC, floating bodies and
    periodic components too short for the reused-cells pass are rejected."""
    import dataclasses
    from paper_2104_00537_amd import cases
    base = cases.dam_break_2d(dp=0.05).params
    P0 = S.make_params(base)
    b, _ = S.sph_batch_describe([P0, P0], [0, 64, 128])
    assert not b.flags & S.SPH_BATCH_GENERAL
    for kw in (dict(kernel=1), dict(viscosity=1, visc_nu=1e-2), dict(ddt=2)):
        ps = [P0, S.make_params(dataclasses.replace(base, **kw))]
        b, _ = S.sph_batch_describe(ps, [0, 64, 128])
        assert b.flags & S.SPH_BATCH_GENERAL, kw
    for kw in (dict(boundary=1), dict(floating=1)):
        ps = [P0, _bad_params(S, **kw)]
        with pytest.raises(S.SphError):
            S.sph_batch_describe(ps, [0, 10, 20])
    # periodic components per slot, long enough for the reused-cells pass
    per = S.make_params(cases.periodic_box(2, shape=(60, 14), periodic=(0,)).params)
    b, _ = S.sph_batch_describe([P0, per], [0, 64, 128])
    assert b.flags & S.SPH_BATCH_PERIODIC
    assert not S.sph_batch_describe([P0, P0], [0, 64, 128])[0].flags & S.SPH_BATCH_PERIODIC
    short = S.make_params(cases.periodic_box(2, shape=(12, 14), periodic=(0,)).params)
    with pytest.raises(S.SphError):   # 4 cells along x: enough for a walk, not for reuse
        S.sph_batch_describe([P0, short], [0, 64, 128])


def test_periodic_params_validate_without_device(S):
    """A periodic component must span exactly its period in whole cells, at
    least 2 cell_div + 1 of them (x: ncell[0] divisible by x_sub); periodic
    cases reject modified DBC, floating bodies, the precision-study arms and
    the batched path."""
    import dataclasses
    from paper_2104_00537_amd import cases
    c = cases.periodic_box(3, periodic=(0, 1), cell_div=2, x_sub=4)
    cp = c.params
    lib = S.lib
    d = C.c_void_p(16)
    st = S.SphState(16, 16, 16, 16, 16, None)
    need = S.sph_workspace_bytes(S.make_params(cp), 1000)

    def interact(p, flags=0):
        return lib.sph_interact(C.byref(p), 1000, C.byref(st), d, d, d, d, None, None, flags, d,
                                need, None)

    P = S.make_params(cp)
    assert P.period[0] > 0 and P.period[1] > 0 and P.period[2] == 0
    # (only calls that are rejected before any device work are made here)
    bad = [dict(period=(cp.period[0] * 1.001, cp.period[1], 0.0)),      # not the grid extent
           dict(period=(cp.period[0], cp.period[1], 0.05)),             # not z's grid extent
           dict(boundary=1), dict(floating=1),
           dict(ncell=(cp.ncell[0] + 1, cp.ncell[1], cp.ncell[2])),     # not divisible by x_sub
           ]
    for kw in bad:
        assert interact(S.make_params(dataclasses.replace(cp, **kw))) == S.SPH_E_ARG, kw
    small = cases.periodic_box(2, shape=(8, 10), periodic=(0,), cell_div=2)
    assert small.params.ncell[0] < 5
    assert interact(S.make_params(small.params)) == S.SPH_E_ARG
    # 6 cells: enough for the cells' own reach of 2, not for the reach of 3 of
    # a walk on reused cells (which would meet a cell twice)
    six = cases.periodic_box(2, shape=(12, 10), periodic=(0,), cell_div=2)
    assert six.params.ncell[0] // six.params.x_sub == 6
    P6 = S.make_params(six.params)
    need6 = S.sph_workspace_bytes(P6, 1000)
    assert lib.sph_interact(C.byref(P6), 1000, C.byref(st), d, d, d, d, None, None,
                            S.SPH_INTERACT_REUSE_CELLS, d, need6, None) == S.SPH_E_ARG
    P6s = S.make_params(dataclasses.replace(six.params, shift_coef=2.0))
    assert lib.sph_shifting(C.byref(P6s), 1000, C.byref(st), d, d, d, None, None,
                            S.SPH_INTERACT_REUSE_CELLS, d, need6, None) == S.SPH_E_ARG
    for flags in (S.SPH_INTERACT_F64, S.SPH_INTERACT_ABS_F32):
        assert interact(P, flags) == S.SPH_E_ARG
    # a batch slot must serve the reused-cells pass too: six cells are short
    with pytest.raises(S.SphError):
        S.sph_batch_describe([S.make_params(cases.dam_break_2d(dp=0.05, cell_div=2).params),
                              P6], [0, 10, 20])


def test_shifting_validates_without_device(S):
    """sph_shifting needs shift_coef > 0; negative or non-finite shifting
    parameters are rejected by every call."""
    import dataclasses
    from paper_2104_00537_amd import cases
    cp = cases.dam_break_2d(dp=0.05).params
    lib = S.lib
    d = C.c_void_p(16)
    st = S.SphState(16, 16, 16, 16, 16, None)
    need = S.sph_workspace_bytes(S.make_params(cp), 1000)

    def shifting(p, ws=need):
        return lib.sph_shifting(C.byref(p), 1000, C.byref(st), d, d, d, None, None, 0, d, ws, None)

    assert shifting(S.make_params(cp)) == S.SPH_E_ARG                 # shift_coef = 0
    ok = dataclasses.replace(cp, shift_coef=2.0)
    assert shifting(S.make_params(ok), ws=need - 1) == S.SPH_E_WORKSPACE
    # flags other than reusing the cells (rejected before any device work)
    for fl in (S.SPH_DIAG_COUNT_F64, S.SPH_INTERACT_ONE_LANE, 1 << 7):
        assert lib.sph_shifting(C.byref(S.make_params(ok)), 1000, C.byref(st), d, d, d, None,
                                None, fl, d, need, None) == S.SPH_E_ARG
    for kw in (dict(shift_coef=-1.0), dict(shift_coef=2.0, shift_fs=-0.5),
               dict(shift_coef=float("inf"))):
        P = S.make_params(dataclasses.replace(cp, **kw))
        assert shifting(P) == S.SPH_E_ARG
        assert lib.sph_interact(C.byref(P), 1000, C.byref(st), d, d, d, d, None, None, 0, d,
                                need, None) == S.SPH_E_ARG
