"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/polyspec.h declares, the ctypes structures match the C
layout, host-side validation rejects bad configurations before touching the
device, and the channel-combination orbits are right."""
import ctypes as C
import itertools
import os
import re
import subprocess
import sys

import pytest

from paper_2505_01231_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polyspec.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ps_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    declared = _declared_functions()
    assert set(declared) == set(L.EXPORTED), declared
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ps_[a-z_0-9]+)\b", out))
    assert set(declared) <= exported


def test_version_and_status_strings():
    lib = L.load()
    assert lib.ps_abi_version() == 1
    for s in range(6):
        assert L.status_string(s).startswith("PS_")


_LAYOUT_PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "polyspec.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("ps_config %zu\n", sizeof(ps_config));
  printf("ps_record %zu\n", sizeof(ps_record));
  printf("ps_output %zu\n", sizeof(ps_output));
  printf("ps_plan_info %zu\n", sizeof(ps_plan_info));
  printf("ps_tuning %zu\n", sizeof(ps_tuning));
  printf("ps_tune_report %zu\n", sizeof(ps_tune_report));
  P(ps_tuning, s3_frame_batch) P(ps_tune_report, cand) P(ps_tune_report, ms)
  P(ps_config, dt) P(ps_config, window) P(ps_config, n_combos4) P(ps_config, combos2) P(ps_config, combos4)
  P(ps_config, interlaced) P(ps_config, estimator) P(ps_config, complex_signal) P(ps_config, s4_shift)
  P(ps_plan_info, grid)
  P(ps_record, n_samples) P(ps_record, dtype) P(ps_output, d_s4_err) P(ps_output, d_s1) P(ps_output, d_s1_err)
  P(ps_plan_info, f_max) P(ps_plan_info, sum_g) P(ps_plan_info, combos4)
  return 0;
}
"""


def test_ctypes_layouts_match_header(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(_LAYOUT_PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                             check=True).stdout.splitlines())
    py = {
        "ps_config": C.sizeof(L.ps_config), "ps_record": C.sizeof(L.ps_record),
        "ps_output": C.sizeof(L.ps_output), "ps_plan_info": C.sizeof(L.ps_plan_info),
        "ps_tuning": C.sizeof(L.ps_tuning), "ps_tune_report": C.sizeof(L.ps_tune_report),
    }
    for k, v in py.items():
        assert int(got[k]) == v, k
    for key, val in got.items():
        if "." in key:
            struct, field = key.split(".")
            assert getattr(getattr(L, struct), field).offset == int(val), key


def test_constants_match_header(tmp_path):
    """Every PS_* constant of the binding has the value the header gives it
    (enumerators and #defines, printed by a C program compiled against the
    header)."""
    text = open(HEADER).read()
    names = sorted(set(re.findall(r"\b(PS_[A-Z0-9_]+)\s*=", text)) |
                   set(re.findall(r"#define\s+(PS_[A-Z0-9_]+)\s+\S", text)))
    py = {n: getattr(L, n) for n in dir(L) if n.startswith("PS_") and isinstance(getattr(L, n), int)}
    assert set(py) <= set(names), sorted(set(py) - set(names))
    src = tmp_path / "consts.c"
    src.write_text('#include <stdio.h>\n#include "polyspec.h"\nint main(void) {\n' +
                   "".join(f'  printf("{n} %lld\\n", (long long)({n}));\n' for n in names) + "  return 0;\n}\n")
    exe = tmp_path / "consts"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = {k: int(v) for k, v in (line.split() for line in subprocess.run(
        [str(exe)], capture_output=True, text=True, check=True).stdout.splitlines())}
    for n, v in py.items():
        assert got[n] == v, (n, got[n], v)


def _cfg(**kw):
    cfg = L.ps_config()
    cfg.struct_size = C.sizeof(L.ps_config)
    cfg.orders = L.PS_ORDER_S2 | L.PS_ORDER_S3 | L.PS_ORDER_S4
    cfg.n_channels = 1
    cfg.frame_len = 256
    cfg.n_freq = 64
    cfg.m = 10
    cfg.dt = 1.0
    cfg.window = L.PS_WIN_HANN
    cfg.window_param = 0.14
    for k, v in kw.items():
        setattr(cfg, k, v)
    return cfg


@pytest.mark.parametrize("kw,status", [
    (dict(frame_len=300, complex_signal=1), L.PS_E_UNSUPPORTED),    # complex: power-of-two frame lengths only
    (dict(frame_len=1536, n_freq=100, frame_len_set=1 << 9), L.PS_E_UNSUPPORTED),  # further lengths: power of two
    (dict(frame_len=255), L.PS_E_UNSUPPORTED),          # below the supported range
    (dict(frame_len=128), L.PS_E_UNSUPPORTED),          # below the supported range
    (dict(frame_len=16384), L.PS_E_UNSUPPORTED),
    (dict(m=3), L.PS_E_INVALID_ARG),                    # S4 needs m >= 4
    (dict(frame_len_set=1 << 14), L.PS_E_INVALID_ARG),   # further frame lengths only 256..8192
    (dict(frame_len_set=1 << 7), L.PS_E_INVALID_ARG),
    (dict(n_freq=65, frame_len=1024, frame_len_set=1 << 8), L.PS_E_INVALID_ARG),   # 65 * 256 / 1024
    (dict(n_freq=64, frame_len=1024, frame_len_set=1 << 9, complex_signal=1), L.PS_E_UNSUPPORTED),
    (dict(n_freq=257, frame_len=1024, frame_len_set=1 << 11), L.PS_E_INVALID_ARG),  # 514 at N = 2048: S3 bound
    (dict(m=2, orders=L.PS_ORDER_S3), L.PS_E_INVALID_ARG),
    (dict(m=1, orders=L.PS_ORDER_S2), L.PS_E_INVALID_ARG),
    (dict(n_freq=66), L.PS_E_INVALID_ARG),              # 2 (Nf - 1) > N/2 with S3
    (dict(n_freq=130, orders=L.PS_ORDER_S2), L.PS_E_INVALID_ARG),
    (dict(n_channels=5), L.PS_E_INVALID_ARG),
    (dict(n_channels=0), L.PS_E_INVALID_ARG),
    (dict(dt=0.0), L.PS_E_INVALID_ARG),
    (dict(dt=float("nan")), L.PS_E_INVALID_ARG),
    (dict(orders=0), L.PS_E_INVALID_ARG),
    (dict(orders=1 << 5), L.PS_E_INVALID_ARG),
    (dict(orders=1), L.PS_E_INVALID_ARG),               # bit 0 is no order
    (dict(orders=L.PS_ORDER_S1 | L.PS_ORDER_S2, m=1), L.PS_E_INVALID_ARG),
    (dict(struct_size=8), L.PS_E_INVALID_ARG),
    (dict(window=7), L.PS_E_INVALID_ARG),
    (dict(window=L.PS_WIN_ACG, window_param=0.0), L.PS_E_INVALID_ARG),
    (dict(precision=9), L.PS_E_INVALID_ARG),
    (dict(schedule=4), L.PS_E_INVALID_ARG),
    (dict(n_freq=0, f_max=-1.0), L.PS_E_INVALID_ARG),
    (dict(interlaced=2), L.PS_E_INVALID_ARG),
    (dict(estimator=3), L.PS_E_INVALID_ARG),
    (dict(estimator=L.PS_EST_C3OPT, m=3), L.PS_E_INVALID_ARG),        # c3^(opt) leaves S4 at m >= 4
    (dict(estimator=L.PS_EST_C3OPT, m=1, orders=L.PS_ORDER_S3), L.PS_E_INVALID_ARG),
    (dict(interlaced=1, schedule=L.PS_SCHED_PER_CHUNK), L.PS_E_UNSUPPORTED),
    (dict(complex_signal=2), L.PS_E_INVALID_ARG),
    (dict(s4_shift=2), L.PS_E_UNSUPPORTED),             # planes need complex_signal
    (dict(complex_signal=1, s4_shift=80), L.PS_E_INVALID_ARG),
    (dict(complex_signal=1, frame_len=8192, n_freq=100), L.PS_E_UNSUPPORTED),
])
def test_plan_validation_rejects_before_device_work(kw, status):
    lib = L.load()
    h = C.c_void_p(123)
    cfg = _cfg(**kw)
    assert lib.ps_plan_create(C.byref(cfg), C.byref(h)) == status
    assert h.value is None
    assert L.last_error()


def test_bad_combinations_rejected():
    lib = L.load()
    arr = (C.c_int8 * 2)(0, 2)
    cfg = _cfg(n_channels=2, orders=L.PS_ORDER_S2, n_combos2=1, combos2=C.cast(arr, C.POINTER(C.c_int8)))
    h = C.c_void_p()
    assert lib.ps_plan_create(C.byref(cfg), C.byref(h)) == L.PS_E_INVALID_ARG
    cfg = _cfg(n_channels=2, orders=L.PS_ORDER_S2, n_combos2=1)   # NULL list with a count
    assert lib.ps_plan_create(C.byref(cfg), C.byref(h)) == L.PS_E_INVALID_ARG


def _orbits(n_ch, order):
    """Independent orbit enumeration: canonical representative = lexicographic
    minimum over the grid-preserving symmetry group of Section 9."""
    if order == 2:
        maps = [lambda c: c, lambda c: (c[1], c[0])]
    elif order == 3:
        maps = [lambda c: c, lambda c: (c[1], c[0], c[2])]
    else:
        maps = [lambda c: c, lambda c: (c[1], c[0], c[3], c[2]), lambda c: (c[2], c[3], c[0], c[1]),
                lambda c: (c[3], c[2], c[1], c[0])]
    reps = []
    for c in itertools.product(range(n_ch), repeat=order):
        if c == min(f(c) for f in maps):
            reps.append(c)
    return reps


@pytest.mark.parametrize("n_ch", [1, 2, 3, 4])
@pytest.mark.parametrize("order", [2, 3, 4])
def test_combination_orbits(n_ch, order):
    from paper_2505_01231_amd.polyspec import enumerate_combos
    got = enumerate_combos(n_ch, order)
    assert got == _orbits(n_ch, order)
    if n_ch == 4:
        assert len(got) == {2: 10, 3: 40, 4: 76}[order]
    # every ordered combination is reachable from exactly one representative
    assert len(set(got)) == len(got)


def test_tuning_calls_reject_null_arguments():
    """The launch-configuration calls validate their arguments on the host."""
    lib = L.load()
    t = L.ps_tuning(8, 0)
    assert lib.ps_plan_get_tuning(None, C.byref(t)) == L.PS_E_INVALID_ARG
    assert lib.ps_plan_set_tuning(None, C.byref(t)) == L.PS_E_INVALID_ARG
    rep = L.ps_tune_report()
    assert lib.ps_plan_autotune(None, None, 0, None, 0, None, 3, None, C.byref(rep)) == L.PS_E_INVALID_ARG
    assert "NULL" in L.last_error()


def test_library_binds_to_torchs_hip_runtime():
    """Loading the library first must not hand torch the system HIP runtime:
    load() imports torch before the library, whose HIP dependency (same
    soname as torch's copy) then resolves to torch's."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2505_01231_amd import _lib\n"
            "assert 'torch' not in sys.modules\n"
            "_lib.load()\n"
            "assert 'torch' in sys.modules\n"
            "maps = open('/proc/self/maps').read()\n"
            "hip = {l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}\n"
            "assert len(hip) == 1, hip\n"
            "import torch, os\n"
            "assert next(iter(hip)).startswith(os.path.dirname(torch.__file__)), hip\n") % ROOT
    subprocess.run([sys.executable, "-c", code], check=True, timeout=300)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and a JSON line
    that says so, before it touches torch or a device."""
    import json
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


@pytest.mark.parametrize("n_ch", [2, 3, 4])
@pytest.mark.parametrize("order", [3, 4])
def test_orbit_quadrants_are_disjoint_pieces(n_ch, order):
    """The positive quadrants of the "every orbit" combinations are disjoint
    pieces of the multichannel polyspectrum: a value is the cumulant of a
    multiset of (channel, frequency) pairs (frequencies summing to zero; for
    real signals conjugation negates every frequency), and no such multiset,
    or its conjugate, is served by two different stored combinations, except on
    the measure-zero lines the cut itself singles out (S4 at k = l, where a
    second pairing of opposite frequencies exists).  So the equivalences of
    Section 9 (e.g. S3_yyx(w) = S3_xyy(M w)) relate points of different
    stored quadrants and cannot remove an orbit from a positive-quadrant
    computation; ps_full_plane applies them when gathering."""
    N = 7
    combos = []
    n = C.c_int32(0)
    assert lib_ok()
    lib = L.load()
    assert lib.ps_enumerate_combos(n_ch, order, None, C.byref(n)) == L.PS_OK
    buf = (C.c_int8 * (n.value * order))()
    assert lib.ps_enumerate_combos(n_ch, order, buf, C.byref(n)) == L.PS_OK
    combos = [tuple(buf[i * order:(i + 1) * order]) for i in range(n.value)]
    seen = {}
    for cb in combos:
        sym = (cb[0] == cb[1]) if order == 3 else (cb[0] == cb[2] and cb[1] == cb[3])
        for k in range(1, N):
            for l in range(1, N):
                if sym and k > l:
                    continue
                if order == 3:
                    pairs = [(cb[0], k), (cb[1], l), (cb[2], -k - l)]
                else:
                    pairs = [(cb[0], k), (cb[1], -k), (cb[2], l), (cb[3], -l)]
                for key in (tuple(sorted(pairs)), tuple(sorted((c, -f) for c, f in pairs))):
                    if key in seen and seen[key][0] != cb:
                        assert order == 4 and k == l and seen[key][1] == seen[key][2] == k, (cb, k, l, seen[key])
                    seen.setdefault(key, (cb, k, l))
    # and every orbit member of a transposition/conjugation class is served
    assert len(combos) == {3: {2: 6, 3: 18, 4: 40}, 4: {2: 7, 3: 27, 4: 76}}[order][n_ch]


def lib_ok():
    return L.load() is not None
