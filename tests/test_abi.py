"""Host-side checks of the C ABI: the library loads, exports every function
the header declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hoomd_mi355x.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set()
    for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(", txt, flags=re.M):
        name = m.group(1)
        if name not in ("if", "while", "sizeof", "defined"):
            names.add(name)
    return names


@pytest.fixture(scope="module")
def hlib():
    from paper_1412_3387_amd import binding, build
    if build.needs_build():
        build.build()
    return binding.lib()


def test_header_declares_the_five_entry_points():
    names = declared_functions()
    for n in ("hoomd_init", "build_nlist", "compute_forces", "step", "pack_ghosts"):
        assert n in names


def test_library_exports_every_declared_symbol(hlib):
    from paper_1412_3387_amd import binding
    names = declared_functions()
    assert names == set(binding.EXPORTS)
    for n in names:
        assert hasattr(hlib, n), n


def test_strerror_and_workspace_sizing(hlib):
    from paper_1412_3387_amd import binding as B
    assert hlib.hoomd_strerror(0) == b"ok"
    assert hlib.hoomd_strerror(5) == b"neighbour row capacity exceeded"
    p = B.ModelParams(precision=B.MIXED).to_c(0.8442)
    box = B.Box()
    for a in range(3):
        box.L[a] = 16.796
        box.periodic[a] = 1
    box.n_local = box.n_cap = 4000
    n1 = hlib.hoomd_workspace_bytes(C.byref(p), 1, C.byref(box))
    assert n1 > 4000 * 4 * p.nlist_cap
    box.n_local = box.n_cap = 8000
    assert hlib.hoomd_workspace_bytes(C.byref(p), 1, C.byref(box)) > n1
    # a box too small for a unique minimum image is rejected
    for a in range(3):
        box.L[a] = 5.0
    assert hlib.hoomd_workspace_bytes(C.byref(p), 1, C.byref(box)) == 0


def test_empty_systems_are_accepted_beside_others_but_not_alone(hlib):
    """A system with no particles (with or without rows) may sit in a batch;
    a context without a single row is rejected."""
    from paper_1412_3387_amd import binding as B
    ps = (B.Params * 3)(*[B.ModelParams(precision=B.MIXED).to_c(0.8442) for _ in range(3)])
    boxes = (B.Box * 3)()
    for b in boxes:
        for a in range(3):
            b.L[a] = 16.796
            b.periodic[a] = 1
    boxes[1].n_local = boxes[1].n_cap = 4000
    boxes[2].n_cap = 100
    assert hlib.hoomd_workspace_bytes(ps, 3, boxes) > 0
    boxes[1].n_local = boxes[1].n_cap = 0
    boxes[2].n_cap = 0
    assert hlib.hoomd_workspace_bytes(ps, 3, boxes) == 0
    assert hlib.hoomd_workspace_bytes(ps, 1, boxes) == 0


def test_init_rejects_bad_arguments_without_device_work(hlib):
    from paper_1412_3387_amd import binding as B
    p = B.ModelParams(precision=B.MIXED).to_c(0.8442)
    box = B.Box()
    for a in range(3):
        box.L[a] = 16.796
        box.periodic[a] = 1
    box.n_local = box.n_cap = 4000
    arr = B.Arrays(None, None, None, None, None)
    h = C.c_void_p()
    assert hlib.hoomd_init(C.byref(h), C.byref(p), 1, C.byref(box), C.byref(arr), 1, 1 << 30, None) == 1
    p.precision = 7
    arr = B.Arrays(1, 1, 1, 1, None)
    assert hlib.hoomd_init(C.byref(h), C.byref(p), 1, C.byref(box), C.byref(arr), 1, 1 << 30, None) == 1
    p.precision = B.MIXED
    assert hlib.hoomd_init(C.byref(h), C.byref(p), 1, C.byref(box), C.byref(arr), 1, 16, None) == 3
    assert hlib.build_nlist(None, 1) == 1 and hlib.step(None, 0, 1, 0) == 1
    assert hlib.compute_forces(None, 0, 0) == 1


def test_tuning_and_check_period_fields_are_validated(hlib):
    """The launch-shape fields accept 0 or the values the library runs
    (hoomd_autotune reports them); the check period must be >= 0 and equal in
    all systems."""
    from paper_1412_3387_amd import binding as B

    def ws(**kw):
        p = B.ModelParams(precision=B.MIXED, **kw).to_c(0.8442)
        box = B.Box()
        for a in range(3):
            box.L[a] = 16.796
            box.periodic[a] = 1
        box.n_local = box.n_cap = 4000
        return hlib.hoomd_workspace_bytes(C.byref(p), 1, C.byref(box))

    assert ws() > 0
    for w, b in ((64, 512), (64, 256), (32, 512), (32, 256)):
        assert ws(tpp_nlist=w, block_nlist=b) > 0
    assert ws(tpp_nlist=4) == 0 and ws(block_nlist=128) == 0 and ws(tpp_nlist=16, block_nlist=512) == 0
    assert ws(tune_period=100) > 0 and ws(tune_period=-1) == 0
    for w in (1, 2, 4, 8, 16):
        assert ws(tpp_force=w, block_force=64 * w) > 0
        assert ws(tpp_force=w, block_force=64 * w + 64) == 0
    assert ws(tpp_force=3) == 0 and ws(tpp_force=32) == 0
    assert ws(block_force=256) == 0  # a block size needs an explicit lane count
    assert ws(check_period=0) > 0 and ws(check_period=5) > 0 and ws(check_period=-1) == 0
    # two systems with different check periods
    ps = (B.Params * 2)(B.ModelParams(check_period=2).to_c(0.8442), B.ModelParams(check_period=3).to_c(0.8442))
    boxes = (B.Box * 2)()
    for b in boxes:
        for a in range(3):
            b.L[a] = 16.796
            b.periodic[a] = 1
        b.n_local = b.n_cap = 4000
    assert hlib.hoomd_workspace_bytes(ps, 2, boxes) == 0
    ps[1].check_period = 2
    assert hlib.hoomd_workspace_bytes(ps, 2, boxes) > 0


def test_layout_struct_matches_header(hlib):
    """hoomd_layout as the binding declares it has the header's fields, in
    order (names parsed from the header)."""
    import re
    from paper_1412_3387_amd import binding as B
    txt = open(HEADER).read()
    body = re.search(r"typedef struct \{([^}]*)\} hoomd_layout;", txt).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\b(\w+)(?:\[\d+\])?;", body)
    assert names == [f[0] for f in B.Layout._fields_]


def test_params_struct_matches_header():
    """hoomd_params as the binding declares it has the header's fields, in
    order (names parsed from the header)."""
    import re
    from paper_1412_3387_amd import binding as B
    txt = open(HEADER).read()
    body = re.search(r"typedef struct \{(.*?)\} hoomd_params;", txt, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in re.findall(r"([^;]+);", body):
        _type, rest = decl.split(None, 1)  # "double eps, sigma" -> eps, sigma
        names += [n.strip() for n in rest.split(",")]
    assert names == [f[0] for f in B.Params._fields_]


def test_force_launch_field_is_validated(hlib):
    """force_launch takes HOOMD_FORCE_AUTO, _SPLIT or _ONE, equal in all
    systems."""
    from paper_1412_3387_amd import binding as B
    boxes = (B.Box * 2)()
    for b in boxes:
        for a in range(3):
            b.L[a] = 16.796
            b.periodic[a] = 1
        b.n_local = b.n_cap = 4000

    def ws(m0, m1):
        ps = (B.Params * 2)(B.ModelParams(force_launch=m0).to_c(0.8442), B.ModelParams(force_launch=m1).to_c(0.8442))
        return hlib.hoomd_workspace_bytes(ps, 2, boxes)

    for m in (B.FORCE_AUTO, B.FORCE_SPLIT, B.FORCE_ONE):
        assert ws(m, m) > 0
    assert ws(-1, -1) == 0 and ws(3, 3) == 0 and ws(B.FORCE_SPLIT, B.FORCE_ONE) == 0


def test_integrator_fields_are_validated(hlib):
    """NVT needs a positive finite set temperature and coupling time and a
    group id >= 0; systems of one thermostat group must share dt, T0 and
    tau; systems with their own thermostats (group 0) need not."""
    from paper_1412_3387_amd import binding as B

    def ws(*kws):
        ps = (B.Params * len(kws))(*[B.ModelParams(**kw).to_c(0.8442) for kw in kws])
        boxes = (B.Box * len(kws))()
        for b in boxes:
            for a in range(3):
                b.L[a] = 16.796
                b.periodic[a] = 1
            b.n_local = b.n_cap = 4000
        return hlib.hoomd_workspace_bytes(ps, len(kws), boxes)

    nvt = dict(integrator=B.NVT, nvt_T0=1.2, nvt_tau=0.5)
    assert ws(nvt) > 0 and ws(dict(integrator=2)) == 0
    assert ws(dict(nvt, nvt_T0=0.0)) == 0 and ws(dict(nvt, nvt_tau=-1.0)) == 0
    assert ws(dict(nvt, nvt_tau=float("inf"))) == 0 and ws(dict(nvt, nvt_group=-1)) == 0
    assert ws(dict(nvt, nvt_group=1), dict(nvt, nvt_group=1)) > 0
    assert ws(dict(nvt, nvt_group=1), dict(nvt, nvt_group=1, nvt_T0=1.0)) == 0
    assert ws(dict(nvt, nvt_group=1), dict(nvt, nvt_group=1, dt=0.004)) == 0
    assert ws(dict(nvt), dict(nvt, nvt_T0=1.0, dt=0.004)) > 0
    assert ws(dict(nvt, nvt_group=1), dict(nvt, nvt_group=2, nvt_T0=1.0)) > 0
