"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and validates plans without touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sipg.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sipg_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_2506_14424_amd import LIB_PATH
    lib = C.CDLL(LIB_PATH)
    names = header_functions()
    assert len(names) >= 17
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_abi_version_and_defaults():
    from paper_2506_14424_amd import _ffi as F
    assert F.lib.sipg_abi_version() == 2
    o = F.SolveOpts()
    F.lib.sipg_solve_opts_default(C.byref(o))
    assert o.rel_tol == 1e-8 and o.cheb_degree == 5 and o.precond_precision == F.F32
    assert o.use_graph == 0 and o.reuse_eigs == 0


def test_plan_counts_and_workspace_on_cpu():
    from paper_2506_14424_amd import Operator
    cfg = W.config("c2", 5)
    op = Operator.from_config(cfg, W.box_vertices(5, 5, 5, 0.1))
    n = 4
    assert op.ndof == 125 * 3 * n ** 3
    assert op.nface == 3 * 6 * 25
    wb_op, wb_all = op.workspace_bytes(False), op.workspace_bytes(True)
    # at least: mu at cell and face points (8+4 bytes), diag + 2 inverses, 9 solver vectors
    assert wb_op >= 12 * (125 * n ** 3 + op.nface * n * n) + 20 * op.ndof
    assert wb_all >= wb_op + 9 * 8 * op.ndof


@pytest.mark.parametrize("kwargs,fragment", [
    (dict(degree=0), "degree"),
    (dict(degree=6), "degree"),
    (dict(alpha=-1.0), "alpha"),
    (dict(penalty=0.0), "penalty"),
    (dict(bc=("D", "D", "X", "D", "D", "D")), None),
    (dict(law={"kind": "sine", "mu": 1.0, "amp": 1.5}), "SINE"),
])
def test_plan_create_rejects_bad_input(kwargs, fragment):
    from paper_2506_14424_amd import Operator, SipgError
    args = dict(nx=2, ny=2, nz=2, degree=2, op="viscous", alpha=1.0, penalty=1.0,
                law=W.sine_law())
    args.update(kwargs)
    with pytest.raises((SipgError, KeyError)) as ei:
        Operator(**args)
    if fragment and isinstance(ei.value, Exception) and hasattr(ei.value, "code"):
        assert ei.value.code == -1 and fragment in str(ei.value)


def test_plan_create_rejects_inverted_cells():
    from paper_2506_14424_amd import Operator, SipgError
    V = W.box_vertices(3, 3, 3, 0.1).reshape(4, 4, 4, 3).copy()
    V[1, 1, 1] = V[2, 2, 2] + 0.05          # fold an interior vertex through its neighbour
    with pytest.raises(SipgError, match="det J"):
        Operator(3, 3, 3, 2, "viscous", 1.0, 1.0, W.sine_law(), V.reshape(-1, 3))


def test_logfield_mode_limit():
    from paper_2506_14424_amd import Operator, SipgError
    law = W.logfield_law(1, 10.0, n_modes=17)
    with pytest.raises(SipgError, match="MAX_MODES"):
        Operator(2, 2, 2, 2, "viscous", 1.0, 1.0, law)


def test_package_has_no_cpu_fallback():
    """The package's compute entry points go through the library only."""
    import paper_2506_14424_amd.operator as opmod
    src = open(opmod.__file__).read()
    assert "oracle" not in src and "numpy.linalg" not in src


def test_package_import_loads_a_single_hip_runtime():
    """Importing the binding before torch must not load a second HIP runtime
    next to torch's (two runtimes in one process cannot share streams or
    device pointers): the package imports torch before opening the library."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_2506_14424_amd\n"
            "libs = set(l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l)\n"
            "print(len(libs))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_picard_entry_points_on_cpu():
    """Defaults, the work size, and the host-side refusals of the Picard
    entry points (no GPU call is made before these checks)."""
    import torch  # noqa: F401
    from paper_2506_14424_amd import Operator, SipgError, _ffi as F
    o = F.PicardOpts()
    F.lib.sipg_picard_opts_default(C.byref(o))
    assert o.rel_tol == 1e-8 and o.abs_tol == 0.0 and o.max_iter == 50 and o.aitken == 1
    cfg = W.config("c3", 3)
    op = Operator.from_config(cfg, W.box_vertices(3, 3, 3, 0.1))
    wb = int(F.lib.sipg_picard_work_bytes(op._h))
    assert wb >= 3 * 8 * op.ndof + 3 * 8 * 512
    dummy = C.c_void_p(256)
    assert F.lib.sipg_update_viscosity(op._h, dummy, None) == -7            # not bound
    rc = F.lib.sipg_picard_solve(op._h, dummy, C.c_void_p(512), C.c_void_p(1024), None, None, None, None)
    assert rc == -7
    assert F.lib.sipg_update_viscosity(op._h, None, None) == -1
    sine = Operator.from_config(W.config("c1"))
    assert F.lib.sipg_update_viscosity(sine._h, dummy, None) == -7


def test_arrays_law_validation_on_cpu():
    """The tabulated viscosity is checked and copied at plan creation; it
    has no multigrid hierarchy."""
    from paper_2506_14424_amd import Operator, SipgError
    cfg = W.config("c1", 2)
    n = cfg["degree"] + 1
    nface = 3 * 3 * 4
    good = {"kind": "arrays", "mu_cell": np.ones((8, n ** 3)), "mu_face": np.ones((nface, n * n))}
    op = Operator(2, 2, 2, cfg["degree"], "viscous", 10.0, 1.0, good)
    assert op.nface == nface
    with pytest.raises(SipgError, match="ARRAYS"):
        Operator(2, 2, 2, cfg["degree"], "viscous", 10.0, 1.0, {"kind": "arrays", "mu_cell": good["mu_cell"],
                                                               "mu_face": -good["mu_face"]})
    with pytest.raises(SipgError, match="multigrid|coarse"):
        op.set_multigrid()


def test_split_step_entry_points_on_cpu():
    """Defaults, the work size, and the host-side refusals of the
    dual-splitting entry points (plans checked before any GPU call)."""
    import torch  # noqa: F401
    from paper_2506_14424_amd import SplitOptions, SplitStep, _ffi as F
    o = F.SplitOpts()
    F.lib.sipg_split_opts_default(C.byref(o))
    assert o.zeta == 1.0 and o.pressure.rel_tol == 1e-8 and o.penalty.cheb_degree == 5
    assert o.pressure.lanczos_steps == o.viscous.lanczos_steps == o.penalty.lanczos_steps == 10
    assert SplitOptions().viscous.lanczos_steps == 10
    law = W.carreau_law(3)
    s = SplitStep(3, 2, 2, 3, 0.01, law, W.box_vertices(3, 2, 2, 0.1))
    assert s.ndof_u == 12 * 3 * 64 and s.ndof_p == 12 * 27
    assert s.work_bytes() >= 5 * 8 * s.ndof_u + 8 * s.ndof_p
    s2 = SplitStep(3, 2, 2, 3, 0.01, law, None, order=2)
    with pytest.raises(ValueError):
        s2._prev(None)                                            # BDF2 needs u_prev
    with pytest.raises(ValueError):
        SplitStep(3, 2, 2, 3, 0.01, law, None, order=3)
    d = C.c_void_p(256)
    assert F.lib.sipg_convective_step(s.vel._h, d, None, None, None, 0.01, C.c_void_p(512), None) == -7  # unbound
    assert F.lib.sipg_pressure_rhs(s.vel._h, s.pres._h, d, d, None, None, None, 0.01, d, None) == -7
    assert F.lib.sipg_wall_load(s.vel._h, d, C.c_void_p(512), None) == -7
    assert F.lib.sipg_update_penalty_factors(s.pen._h, d, 0.01, 1.0, None) == -7
    rc = F.lib.sipg_split_step(s.vel._h, s.pres._h, s.pen._h, d, None, None, None, 0.01, d, d, d, None, None, None)
    assert rc == -7
    # wrong plans: Neumann sides on the velocity, pressure of the wrong degree
    from paper_2506_14424_amd import Operator
    bad = Operator(3, 2, 2, 3, "viscous", 100.0, 1.0, law, None, ("D", "N", "D", "D", "D", "D"))
    assert F.lib.sipg_convective_step(bad._h, d, None, None, None, 0.01, C.c_void_p(512), None) == -1
    assert "no-slip" in F.lib.sipg_last_error().decode()
    assert F.lib.sipg_convective_step(None, d, None, None, None, 0.01, d, None) == -1
    assert s.wall_count() == 2 * (2 * 2 + 3 * 2 + 3 * 2)
    with pytest.raises(ValueError):
        SplitStep(3, 2, 2, 3, 0.01, W.sine_law(1.0, 0.5))


def kernel_scratch_bytes(lib_path):
    """Per-lane scratch (private segment) of every kernel in the library's
    gfx950 code objects, from the code-object metadata notes."""
    import shutil
    import subprocess
    import tempfile
    tools = "/opt/rocm/llvm/bin"
    need = [os.path.join(tools, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]
    if not all(shutil.which(t) for t in need):
        pytest.skip("ROCm LLVM tools not found")
    out = {}
    with tempfile.TemporaryDirectory() as d:
        fat = os.path.join(d, "fat.bin")
        subprocess.run([need[0], f"--dump-section=.hip_fatbin={fat}", lib_path, os.path.join(d, "lib.o")],
                       check=True, capture_output=True)
        data = open(fat, "rb").read()
        offs = [m.start() for m in re.finditer(b"__CLANG_OFFLOAD_BUNDLE__", data)] + [len(data)]
        for i in range(len(offs) - 1):
            b, co = os.path.join(d, f"b{i}.bin"), os.path.join(d, f"c{i}.o")
            open(b, "wb").write(data[offs[i]:offs[i + 1]])
            subprocess.run([need[1], "--unbundle", "--type=o", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                            f"--input={b}", f"--output={co}"], check=True, capture_output=True)
            notes = subprocess.run([need[2], "--notes", co], check=True, capture_output=True, text=True).stdout
            if "amdhsa.kernels:" not in notes:
                continue
            body = re.split(r"\namdhsa\.", notes[notes.index("amdhsa.kernels:"):])[0]
            for k in re.split(r"\n  - ", body)[1:]:
                name = re.search(r"\.name:\s+(\S+)", k).group(1)
                out[name] = int(re.search(r"\.private_segment_fixed_size:\s+(\d+)", k).group(1))
    return out


def test_hot_kernels_use_no_scratch():
    """The splitting-step kernels and the FP64/FP32 apply instances up to
    n = 5 keep everything in registers and LDS: a kernel argument copied to
    scratch for runtime indexing (or a spill) shows up here at build time."""
    from paper_2506_14424_amd import LIB_PATH
    scratch = kernel_scratch_bytes(LIB_PATH)
    split = {k: v for k, v in scratch.items() if re.search(r"k_split_|k_pen_factors|k_wall_load", k)}
    assert len(split) == 28, sorted(split)        # 7 kernels (ppe right-hand side: 2 BDF orders) x n = 3..6
    assert not {k: v for k, v in split.items() if v}
    apply = {k: v for k, v in scratch.items() if re.match(r"_ZN4sipg7k_applyILi[2-5]E", k)}
    assert len(apply) >= 40
    assert not {k: v for k, v in apply.items() if v}
