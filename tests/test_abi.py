"""The C ABI library on the CPU: it loads, exports every symbol include/lb.h
declares, and rejects bad arguments before touching a device (no compute
calls are made here)."""

import ctypes
import os
import re

import pytest

from paper_1405_6162_amd import lb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lb.h")


def _declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(lb_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    return lb.load()


# The argument checks below hand the library made-up device addresses; a
# check that wrongly let one through would queue a kernel on them.  Without a
# GPU that launch only fails; with one it would fault, so they run GPU-less.
no_device = pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="fake device pointers: run where no GPU is visible")


def test_header_declares_the_boundary():
    syms = _declared_symbols()
    for name in ("lb_create", "lb_init_equilibrium", "lb_collide", "lb_propagate", "lb_step",
                 "lb_moments", "lb_destroy"):
        assert name in syms
    assert set(syms) == set(lb._SIGNATURES), "binding and header disagree"


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_symbols():
        assert hasattr(lib, name), name


def test_constants_match_header():
    text = open(HEADER).read()
    for name in ("LB_OK", "LB_EINVAL", "LB_ENOMEM", "LB_EDEVICE", "LB_ENOTSUP", "LB_ERANGE", "LB_NOALLOC_MAX_BLOCKS",
                 "LB_SINGLE", "LB_BGK", "LB_TRT", "LB_MRT",
                 "LB_BINARY", "LB_F64", "LB_F32", "LB_F16", "LB_K_COLLIDE", "LB_K_PHI", "LB_STEP_AUTO",
                 "LB_STEP_MARCH", "LB_STEP_TWO_PASS",
                 "LB_K_STREAM", "LB_K_ADJOINT", "LB_K_OTHER"):
        m = re.search(r"#define\s+%s\s+\(?(-?\d+)\)?" % name, text)
        assert m, name
        assert int(m.group(1)) == getattr(lb, name), name


def test_params_struct_layout(tmp_path):
    """ctypes layout of lb_params equals the C compiler's."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [f[0] for f in lb.lb_params._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lb.h"\nint main(void){\n'
                   + 'printf("%zu\\n", sizeof(lb_params));\n'
                   + "".join('printf("%%zu\\n", offsetof(lb_params, %s));\n' % f for f in fields)
                   + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert out[0] == ctypes.sizeof(lb.lb_params)
    assert out[1:] == [getattr(lb.lb_params, f).offset for f in fields]


def _ws(params):
    n = ctypes.c_size_t(0)
    rc = lb._lib.lb_workspace_bytes(ctypes.byref(params), ctypes.byref(n))
    return rc, n.value


def test_workspace_bytes_valid(lib):
    for model in (lb.LB_SINGLE, lb.LB_BINARY):
        for storage in (lb.LB_F64, lb.LB_F32, lb.LB_F16):
            rc, n = _ws(lb.make_params(16, 16, 16, model=model, storage=storage))
            assert rc == lb.LB_OK
            es = {lb.LB_F64: 8, lb.LB_F32: 4, lb.LB_F16: 2}[storage]
            ndist = 2 if model == lb.LB_SINGLE else 4
            assert n >= ndist * 19 * 16 ** 3 * es
            assert n % 4096 == 0


@pytest.mark.parametrize("change", [
    dict(nx=0), dict(ny=-1), dict(nz=0), dict(model=2), dict(storage=3), dict(tau_f=0.5),
    dict(tau_f=float("nan")), dict(model=1, mobility=0.0), dict(model=1, gamma=-1.0),
    dict(model=1, kappa=-0.1), dict(nx=2048, ny=2048, nz=1024), dict(rho0=float("inf")),
])
def test_bad_parameters_rejected(lib, change):
    kw = dict(nx=8, ny=8, nz=8)
    kw.update(change)
    p = lb.make_params(**kw)
    rc, _ = _ws(p)
    assert rc == lb.LB_EINVAL
    ctx = ctypes.c_void_p()
    assert lib.lb_create(ctypes.byref(p), ctypes.c_void_p(4096), 1 << 30, None, ctypes.byref(ctx)) == lb.LB_EINVAL
    assert not ctx.value


def test_collision_values(lib):
    assert _ws(lb.make_params(4, 4, 4, collision=lb.LB_TRT, tau_minus=1.2))[0] == lb.LB_OK
    assert _ws(lb.make_params(4, 4, 4, collision=lb.LB_TRT, tau_minus=0.5))[0] == lb.LB_EINVAL
    assert _ws(lb.make_params(4, 4, 4, collision=3))[0] == lb.LB_EINVAL
    mrt = dict(collision=lb.LB_MRT, tau_minus=1.1, tau_bulk=1.4, tau_ghost_even=0.9, tau_ghost_odd=1.2)
    assert _ws(lb.make_params(4, 4, 4, **mrt))[0] == lb.LB_OK
    for bad in ("tau_bulk", "tau_ghost_even", "tau_ghost_odd", "tau_minus"):
        assert _ws(lb.make_params(4, 4, 4, **dict(mrt, **{bad: 0.5})))[0] == lb.LB_EINVAL, bad
    assert _ws(lb.make_params(4, 4, 4, model=lb.LB_BINARY, **mrt))[0] == lb.LB_OK
    assert _ws(lb.make_params(4, 4, 4, model=lb.LB_BINARY, collision=lb.LB_TRT, tau_minus=1.2))[0] == lb.LB_OK
    p = lb.make_params(4, 4, 4)
    p.binary_step = 3
    assert _ws(p)[0] == lb.LB_EINVAL
    for step in (lb.LB_STEP_AUTO, lb.LB_STEP_MARCH, lb.LB_STEP_TWO_PASS):
        assert _ws(lb.make_params(4, 4, 4, model=lb.LB_BINARY, binary_step=step))[0] == lb.LB_OK


def test_vvl_values(lib):
    for v, ok in ((0, True), (1, True), (2, True), (4, True), (3, False), (8, False), (-1, False)):
        p = lb.make_params(4, 4, 4, vvl=v)
        assert (_ws(p)[0] == lb.LB_OK) == ok, v


@no_device
def test_create_checks_workspace_without_device_work(lib):
    p = lb.make_params(6, 5, 4, model=lb.LB_BINARY)
    _, need = _ws(p)
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)          # never dereferenced: no call below queues work
    assert lib.lb_create(ctypes.byref(p), fake, need - 1, None, ctypes.byref(ctx)) == lb.LB_ENOMEM
    assert lib.lb_create(ctypes.byref(p), ctypes.c_void_p((1 << 20) + 8), need, None,
                         ctypes.byref(ctx)) == lb.LB_EINVAL           # not 256-byte aligned
    assert lib.lb_create(ctypes.byref(p), None, need, None, ctypes.byref(ctx)) == lb.LB_EINVAL
    assert lib.lb_create(ctypes.byref(p), fake, need, None, ctypes.byref(ctx)) == lb.LB_OK
    try:
        assert lib.lb_step(ctx, -1) == lb.LB_EINVAL
        assert lib.lb_step(ctx, 0) == lb.LB_OK                     # no-op
        assert lib.lb_set_tau(ctx, 0.5) == lb.LB_EINVAL
        assert lib.lb_set_tau(ctx, 0.9) == lb.LB_OK
        assert lib.lb_init_equilibrium(ctx, fake, fake, None) == lb.LB_EINVAL   # binary needs phi
        assert lib.lb_get_state(ctx, fake, None) == lb.LB_EINVAL               # binary needs g
        assert lib.lb_set_state(ctx, fake, None) == lb.LB_EINVAL
        assert lib.lb_conserved_sums(ctx, None) == lb.LB_EINVAL
        assert lib.lb_adjoint_step(ctx, fake, 0, fake, ctypes.c_void_p((1 << 21)), fake) == lb.LB_ENOTSUP
        assert lib.lb_step_record(ctx, -1, fake, None) == lb.LB_EINVAL
        assert lib.lb_step_record(ctx, 0, None, None) == lb.LB_OK                # no-op
        # binary adjoint: aliasing and missing arguments are refused before any launch
        a, b2, c2, d2 = (ctypes.c_void_p((k + 2) << 20) for k in range(4))
        e2 = ctypes.c_void_p(7 << 20)
        assert lib.lb_adjoint_step_binary(ctx, fake, a, None, 0, b2, c2, b2, d2, fake) == lb.LB_EINVAL
        assert lib.lb_adjoint_step_binary(ctx, fake, a, None, 0, b2, c2, d2, d2, fake) == lb.LB_EINVAL
        assert lib.lb_adjoint_step_binary(ctx, fake, a, None, 0, b2, c2, d2, None, fake) == lb.LB_EINVAL
        assert lib.lb_adjoint_step_binary(ctx, fake, a, e2, 0, b2, c2, e2, d2, fake) == lb.LB_EINVAL  # phi aliased
        assert lib.lb_adjoint_init_binary(ctx, fake, fake, fake, fake, fake, None, fake, fake, fake) == lb.LB_EINVAL
        # segment sweeps: bad lengths, missing records and overlapping arrays are refused before any launch
        n = 6 * 5 * 4
        w = ctypes.c_void_p(9 << 20)
        seg = lib.lb_adjoint_segment_binary
        assert seg(ctx, fake, a, b2, None, 0, c2, d2, w, e2) == lb.LB_EINVAL               # length 0
        assert seg(ctx, fake, a, None, None, 2, c2, d2, w, e2) == lb.LB_EINVAL             # no records
        assert seg(ctx, fake, a, b2, None, 1, c2, c2, w, e2) == lb.LB_EINVAL               # lf == lg
        inside_work = ctypes.c_void_p((9 << 20) + 8 * 19 * n)                             # work holds 38 N
        assert seg(ctx, fake, a, b2, None, 1, c2, inside_work, w, e2) == lb.LB_EINVAL
        inside_post = ctypes.c_void_p(b2.value + 8 * 38 * n)                              # post holds 2 x 38 N
        assert seg(ctx, fake, a, b2, None, 3, inside_post, d2, w, e2) == lb.LB_EINVAL
        assert seg(ctx, fake, a, b2, None, 1, c2, d2, w, c2) == lb.LB_EINVAL               # grads inside lf
        assert seg(ctx, fake, a, b2, None, 1, c2, d2, w, None) == lb.LB_EINVAL
        assert lib.lb_adjoint_segment(ctx, fake, None, 1, c2, d2, e2) == lb.LB_ENOTSUP     # binary context
        # set_params: physics may change, layout and deviation references may not
        q = lb.make_params(6, 5, 4, model=lb.LB_BINARY, kappa=0.05, mobility=0.3)
        assert lib.lb_set_params(ctx, ctypes.byref(q)) == lb.LB_OK
        for bad in (lb.make_params(6, 5, 5, model=lb.LB_BINARY), lb.make_params(6, 5, 4, model=lb.LB_BINARY, rho0=2.0),
                    lb.make_params(6, 5, 4, model=lb.LB_BINARY, storage=lb.LB_F32),
                    lb.make_params(6, 5, 4, model=lb.LB_BINARY, mobility=-1.0)):
            assert lib.lb_set_params(ctx, ctypes.byref(bad)) == lb.LB_EINVAL
        assert lib.lb_profile_mask(ctx, 1 << (lb.LB_K_OTHER + 1)) == lb.LB_EINVAL      # no such kernel class
        assert lib.lb_profile_mask(ctx, 0) == lb.LB_OK                                  # stop: no device work
        ms, n = ctypes.c_double(), ctypes.c_int64()
        assert lib.lb_kernel_times(ctx, 7, ctypes.byref(ms), ctypes.byref(n)) == lb.LB_EINVAL
        assert lib.lb_kernel_times(ctx, lb.LB_K_COLLIDE, ctypes.byref(ms), ctypes.byref(n)) == lb.LB_OK
        assert n.value == 0
    finally:
        assert lib.lb_destroy(ctx) == lb.LB_OK


@no_device
def test_stream_copy_refusals(lib):
    """lb_stream_copy checks its arguments before any launch: NULL, 16-byte
    alignment of both pointers and of the size, overlapping ranges."""
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20)
    assert lib.lb_stream_copy(a, b, 0, None) == lb.LB_OK                       # no-op
    assert lib.lb_stream_copy(None, b, 16, None) == lb.LB_EINVAL
    assert lib.lb_stream_copy(a, None, 16, None) == lb.LB_EINVAL
    assert lib.lb_stream_copy(ctypes.c_void_p((1 << 20) + 8), b, 16, None) == lb.LB_EINVAL
    assert lib.lb_stream_copy(a, ctypes.c_void_p((2 << 20) + 4), 16, None) == lb.LB_EINVAL
    assert lib.lb_stream_copy(a, b, 24, None) == lb.LB_EINVAL
    assert lib.lb_stream_copy(a, ctypes.c_void_p((1 << 20) + 16), 32, None) == lb.LB_EINVAL   # overlap
    assert lib.lb_stream_copy(ctypes.c_void_p((1 << 20) + 16), a, 32, None) == lb.LB_EINVAL


@no_device
def test_single_model_rejects_phi(lib):
    p = lb.make_params(4, 4, 4)
    _, need = _ws(p)
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)
    assert lib.lb_create(ctypes.byref(p), fake, need, None, ctypes.byref(ctx)) == lb.LB_OK
    try:
        assert lib.lb_moments(ctx, None, None, fake) == lb.LB_EINVAL
        assert lib.lb_moments(ctx, None, None, None) == lb.LB_OK    # nothing requested
        assert lib.lb_get_state(ctx, fake, fake) == lb.LB_EINVAL
        assert lib.lb_adjoint_step(ctx, fake, 1, fake, fake, fake) == lb.LB_EINVAL   # lam_n aliases
        assert lib.lb_step_record(ctx, 3, None, None) == lb.LB_EINVAL
        assert lib.lb_step_record(ctx, 0, None, fake) == lb.LB_EINVAL          # phi: binary only
        a = [ctypes.c_void_p((k + 2) << 20) for k in range(7)]
        assert lib.lb_adjoint_step_binary(ctx, a[0], a[1], None, 0, a[2], a[3], a[4], a[5], a[6]) == lb.LB_ENOTSUP
        assert lib.lb_adjoint_init_binary(ctx, *a, fake, fake, fake) == lb.LB_ENOTSUP
        n19 = 19 * 4 * 4 * 4
        assert lib.lb_adjoint_segment(ctx, a[0], None, 0, a[1], a[2], a[3]) == lb.LB_EINVAL   # length 0
        assert lib.lb_adjoint_segment(ctx, a[0], None, 2, a[1], a[2], a[3]) == lb.LB_EINVAL   # no records
        assert lib.lb_adjoint_segment(ctx, a[0], None, 1, a[1], a[1], a[3]) == lb.LB_EINVAL   # work == lam
        assert lib.lb_adjoint_segment(ctx, a[0], None, 1, a[1], a[2], a[0]) == lb.LB_EINVAL   # domega is f0
        lam_in_post = ctypes.c_void_p(a[4].value + 8 * n19)                                   # post holds 2 x 19 N
        assert lib.lb_adjoint_segment(ctx, a[0], a[4], 3, lam_in_post, a[2], a[3]) == lb.LB_EINVAL
        assert lib.lb_adjoint_segment_binary(ctx, a[0], a[1], None, None, 1, a[2], a[3], a[4], a[5]) == lb.LB_ENOTSUP
    finally:
        assert lib.lb_destroy(ctx) == lb.LB_OK


@no_device
def test_collision_support_of_the_adjoint_calls(lib):
    """The adjoint calls take every collision but need FP64 storage: a
    binary MRT lattice in FP32 gets LB_ENOTSUP before any launch."""
    fake = [ctypes.c_void_p((k + 2) << 20) for k in range(8)]
    p = lb.make_params(6, 5, 4, model=lb.LB_BINARY, storage=lb.LB_F32, collision=lb.LB_MRT, tau_minus=1.2)
    _, need = _ws(p)
    ctx = ctypes.c_void_p()
    assert lib.lb_create(ctypes.byref(p), ctypes.c_void_p(1 << 20), need, None, ctypes.byref(ctx)) == lb.LB_OK
    try:
        assert lib.lb_adjoint_step_binary(ctx, *fake[:3], 0, *fake[3:7], fake[7]) == lb.LB_ENOTSUP
        assert lib.lb_adjoint_segment_binary(ctx, fake[0], fake[1], None, None, 1, *fake[2:6]) == lb.LB_ENOTSUP
    finally:
        assert lib.lb_destroy(ctx) == lb.LB_OK


@no_device
def test_noalloc_sums_refusals(lib):
    """lb_conserved_sums_noalloc checks its arguments and the size of its
    fixed scratch before it looks up the device array or launches."""
    fake = [ctypes.c_void_p((k + 2) << 20) for k in range(3)]
    p = lb.make_params(8, 8, 8, model=lb.LB_BINARY)
    assert lib.lb_conserved_sums_noalloc(None, fake[0], fake[1], fake[2], None) == lb.LB_EINVAL
    assert lib.lb_conserved_sums_noalloc(ctypes.byref(p), None, fake[1], fake[2], None) == lb.LB_EINVAL
    assert lib.lb_conserved_sums_noalloc(ctypes.byref(p), fake[0], None, fake[2], None) == lb.LB_EINVAL   # g: binary
    assert lib.lb_conserved_sums_noalloc(ctypes.byref(p), fake[0], fake[1], None, None) == lb.LB_EINVAL
    s = lb.make_params(8, 8, 8)
    assert lib.lb_conserved_sums_noalloc(ctypes.byref(s), fake[0], fake[1], fake[2], None) == lb.LB_EINVAL  # no g
    bad = lb.make_params(8, 8, 8, tau_f=0.4)
    assert lib.lb_conserved_sums_noalloc(ctypes.byref(bad), fake[0], None, fake[2], None) == lb.LB_EINVAL
    # ceil(64/64) * ceil(4/4) * nz blocks: one past the fixed array
    big = lb.make_params(64, 4, lb.LB_NOALLOC_MAX_BLOCKS + 1)
    assert lib.lb_conserved_sums_noalloc(ctypes.byref(big), fake[0], None, fake[2], None) == lb.LB_ERANGE


def test_null_handles(lib):
    assert lib.lb_destroy(None) == lb.LB_OK
    assert lib.lb_step(None, 1) == lb.LB_EINVAL
    assert lib.lb_collide(None) == lb.LB_EINVAL
    assert lib.lb_propagate(None) == lb.LB_EINVAL
    assert lib.lb_workspace_bytes(None, None) == lb.LB_EINVAL
    assert lb.lb_strerror(lb.LB_ENOMEM) == "workspace too small"
    assert lb.lb_strerror(12345) == "unknown status"


def test_readme_example_compiles_and_runs_on_the_c_reference(tmp_path):
    """The C block of README.md, compiled as written, runs against the C
    reference library (the same header on host memory; host calloc/free
    stand in for hipMalloc/hipFree): the parameters it builds are accepted
    and the 100 steps it runs conserve mass and the order parameter."""
    import shutil
    import subprocess
    from oracle import build as obuild
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(obuild.LIB):
        obuild.build()
    text = open(os.path.join(ROOT, "README.md")).read()
    block = re.search(r"```c\n(.*?)```", text, flags=re.S).group(1)
    src = tmp_path / "readme_example.c"
    src.write_text(
        "#include <stdio.h>\n#include <stdlib.h>\n#include \"lb.h\"\n"
        "static int hipMalloc(void** p, size_t n) { *p = calloc(1, n); return *p == NULL; }\n"
        "static int hipFree(void* p) { free(p); return 0; }\n"
        "int main(void) {\n"
        "    const int nx = 6, ny = 5, nz = 4;\n    void* stream = NULL;\n"
        "    const size_t N = (size_t)nx * ny * nz;\n"
        "    double *rho = malloc(N * sizeof(double)), *u = calloc(3 * N, sizeof(double)),\n"
        "           *phi = malloc(N * sizeof(double));\n"
        "    double m0 = 0.0, p0 = 0.0, m1 = 0.0, p1 = 0.0;\n"
        "    for (size_t s = 0; s < N; ++s) { rho[s] = 1.0 + 0.001 * (double)(s % 5);\n"
        "        phi[s] = 0.01 * ((double)(s % 7) - 3.0); m0 += rho[s]; p0 += phi[s]; }\n"
        + block +
        "    for (size_t s = 0; s < N; ++s) { m1 += rho[s]; p1 += phi[s]; }\n"
        "    printf(\"%.17g %.17g %.17g %.17g\\n\", m0, m1, p0, p1);\n"
        "    free(rho); free(u); free(phi);\n    return 0;\n}\n")
    exe = tmp_path / "readme_example"
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-L", os.path.dirname(obuild.LIB), "-llb_oracle", "-Wl,-rpath," + os.path.dirname(obuild.LIB),
                    "-o", str(exe)], check=True)
    m0, m1, p0, p1 = (float(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True, timeout=60).stdout.split())
    assert m1 == pytest.approx(m0, rel=1e-12) and m0 > 100
    assert p1 == pytest.approx(p0, abs=1e-12)


def _round_up(n, a=4096):
    return (n + a - 1) // a * a


@pytest.mark.parametrize("n,storage,blocked", [
    (256, lb.LB_F64, True),      # 2.55 GB per buffer
    (320, lb.LB_F64, False),     # 4.98 GB: 8-byte elements take byte offsets, below 4 GiB only
    (384, lb.LB_F32, True),      # 4.30 GB: 4-byte elements are addressed by element
    (384, lb.LB_F16, True),      # 2.15 GB
])
def test_state_layout_choice(lib, n, storage, blocked):
    """The workspace of a binary lattice holds four distribution buffers,
    phi and the block partials; its size shows which state layout the
    library chose: 64-site blocks of all 19 directions (no padding between
    directions) or a structure of arrays (each direction padded to 4 KiB plus
    9472 bytes)."""
    rc, got = _ws(lb.make_params(n, n, n, model=lb.LB_BINARY, storage=storage))
    assert rc == lb.LB_OK
    es = {lb.LB_F64: 8, lb.LB_F32: 4, lb.LB_F16: 2}[storage]
    N = n ** 3
    xblocks = -(-n // 64)
    if blocked:
        dist = _round_up(n * n * xblocks * 19 * 64 * es)
    else:
        dist = _round_up((_round_up(N * es) + 9472) * 19)
    phi = _round_up(N * (8 if storage == lb.LB_F64 else 4))
    partial = _round_up(xblocks * (-(-n // 4)) * n * 16 * 8)
    assert got == 4 * dist + phi + partial
