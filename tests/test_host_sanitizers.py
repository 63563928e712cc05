"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU).

* The library's host runtime (lbm.hip, lbm3d.hip, hbm_copy.hip compiled for the host only, with
  the sanitizers on the host side) linked into tests/native/host_abi_driver.cpp: parameter checks
  on randomly corrupted parameter sets, footprints, tile shapes, the equation-of-state solves
  (compared with the regular build bit for bit), error strings, and every context and batch call
  given invalid arguments.  Leak detection is off for this program: the HIP runtime it links
  keeps allocations of its own until exit.
* The exact division by per-instance constants that the step kernel uses for tile positions
  (tests/native/fastdiv_check.cpp), against integer division on every divisor up to 70 000 and on
  large ones, at and around multiples and at the extremes.
* Both oracles compiled into tests/native/oracle_driver.c and oracle3d_driver.c, run over every
  boundary kind and thermal lattice on small grids, leak detection on; their results equal the
  regular oracle builds bit for bit (same source, no contraction, only the optimisation level
  differs)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2205_00686_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]
GCC_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r


@pytest.fixture(scope="module")
def build_dir(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    return tmp_path_factory.mktemp("sanitized")


@pytest.fixture(scope="module")
def host_driver(build_dir):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    objs = []
    common = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *HOST_SAN, "-I" + os.path.join(ROOT, "include")]
    for name in ("lbm.hip", "lbm3d.hip", "hbm_copy.hip"):
        obj = str(build_dir / (name + ".o"))
        # host code only: the device code is not needed by anything the driver calls
        _run([HIPCC, "--offload-host-only", "-fgpu-rdc", "-x", "hip", *common, "-c", os.path.join(CSRC, name), "-o", obj])
        objs.append(obj)
    drv = str(build_dir / "host_abi_driver.o")
    _run([HIPCC, *common, "-c", os.path.join(NATIVE, "host_abi_driver.cpp"), "-o", drv])
    exe = str(build_dir / "host_abi_driver")
    _run([HIPCC, "-fgpu-rdc", "--offload-arch=gfx950", *HOST_SAN, "-o", exe, drv, *objs,
          "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"])
    return exe


def test_host_runtime_under_sanitizers(host_driver):
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    r = _run([host_driver], env=env, timeout=600)
    lines = r.stdout.split("\n")
    assert "ok" in lines
    import paper_2205_00686_amd as lbm
    from workloads import Params

    base = Params()
    Tc = lbm.critical_temperature(base)
    rows = [list(map(float, ln.split()[1:])) for ln in lines if ln.startswith("coexistence")]
    assert len(rows) == 8
    for ratio, rl, rg, ps in rows:
        assert (rl, rg, ps) == tuple(lbm.coexistence(base, ratio * Tc))


def test_fast_division_is_exact(build_dir):
    """The multiply-high division the step kernel uses for tile positions, compiled for the host
    from the same header, against integer division."""
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(build_dir / "fastdiv_check")
    _run([HIPCC, "--offload-host-only", "-x", "hip", "-std=c++17", "-O1", "-g", *HOST_SAN,
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-o", exe, os.path.join(NATIVE, "fastdiv_check.cpp")])
    r = _run([exe], env=dict(ENV, ASAN_OPTIONS="halt_on_error=1"), timeout=300)
    assert "mismatches 0" in r.stdout, r.stdout


def _gcc(build_dir, src, name):
    exe = str(build_dir / name)
    _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", *GCC_SAN,
          "-o", exe, os.path.join(NATIVE, src), "-lm"])
    return exe


def _cases2d(orc):
    from workloads import Params, boiling, droplet, evaporation, heated_droplet

    base = Params()
    Tc = orc.Tc(base)
    rl, rg, ps = orc.maxwell(base, 0.86 * Tc)
    out = [("periodic droplet", droplet(Tc, rl, rg, nx=40, ny=32, R=8.0), 60),
           ("walls, gravity, hot spot", boiling(Tc, rl, rg, nx=48, ny=40, gravity=5e-5, hot_width=5.0, seed=3), 60),
           ("open top", boiling(Tc, rl, rg, nx=40, ny=36, gravity=5e-5, hot_width=5.0, seed=4, open_top=1), 60),
           ("Dirichlet box", evaporation(Tc, rl, rg, nx=36, ny=30, R=7.0), 60),
           ("heated droplet, open top", heated_droplet(Tc, rl, rg, nx=44, ny=30, R=8.0, gy=-5e-5), 60),
           ("tiny 3x3", droplet(Tc, rl, rg, nx=3, ny=3, R=1.0), 20),
           ("ragged 5x17", boiling(Tc, rl, rg, nx=5, ny=17, gravity=5e-5, hot_width=2.0, seed=5), 30)]
    w = droplet(Tc, rl, rg, nx=30, ny=26, R=6.0)
    w.params.thermal_q = 9
    out.append(("D2Q9 thermal lattice", w, 40))
    w = droplet(Tc, rl, rg, nx=30, ny=26, R=6.0)
    w.params.flags = orc.FREEZE_FLOW | orc.NO_S
    w.ux[:] = 0.03
    out.append(("test flags", w, 40))
    w = droplet(Tc, rl, rg, nx=30, ny=26, R=6.0)
    w.params.flags = orc.BGK
    out.append(("D2Q5 BGK", w, 40))
    return out


def test_oracle_under_sanitizers(build_dir, orc):
    exe = _gcc(build_dir, "oracle_driver.c", "oracle_driver")
    for label, w, steps in _cases2d(orc):
        c = orc._params_struct(w.params)
        n = w.params.nx * w.params.ny
        inp, outp = build_dir / "in2.bin", build_dir / "out2.bin"
        with open(inp, "wb") as fh:
            fh.write(bytes(c))
            fh.write(np.int64(steps).tobytes())
            for a in (w.rho, w.ux, w.uy, w.T):
                fh.write(np.ascontiguousarray(a, dtype=np.float64).tobytes())
        _run([exe, str(inp), str(outp)], env=dict(ENV, ASAN_OPTIONS="halt_on_error=1"), timeout=300)
        raw = np.fromfile(outp, dtype=np.uint8)
        status = int(raw[:4].view(np.int32)[0])
        vals = raw[4:].view(np.float64)
        o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
        o.step(steps)
        exp_fields = np.concatenate([a.ravel() for a in o.fields()])
        f, g, h = o.state()
        exp_state = np.concatenate([f.ravel(), g.ravel(), h.ravel()])
        print(f"[case] sanitized oracle: {label}, {steps} steps", flush=True)
        assert status == 0, label
        assert np.array_equal(vals[:4 * n], exp_fields), label
        assert np.array_equal(vals[4 * n:], exp_state), label


def test_3d_oracle_under_sanitizers(build_dir, orc):
    from oracle import o3d
    from workloads import Params, droplet3d, evaporation3d

    exe = _gcc(build_dir, "oracle3d_driver.c", "oracle3d_driver")
    base = Params()  # the same equation of state as in three dimensions
    Tc = orc.Tc(base)
    rl, rg, _ = orc.maxwell(base, 0.86 * Tc)
    cases = [("3-D droplet", droplet3d(Tc, rl, rg, n=14, R=4.0), 20),
             ("3-D Dirichlet box", evaporation3d(Tc, rl, rg, n=12, R=3.5), 20)]
    for label, w, steps in cases:
        c = o3d._struct(w.params)
        n = w.params.nx * w.params.ny * w.params.nz
        inp, outp = build_dir / "in3.bin", build_dir / "out3.bin"
        with open(inp, "wb") as fh:
            fh.write(bytes(c))
            fh.write(np.int64(steps).tobytes())
            for a in (w.rho, w.ux, w.uy, w.uz, w.T):
                fh.write(np.ascontiguousarray(a, dtype=np.float64).tobytes())
        _run([exe, str(inp), str(outp)], env=dict(ENV, ASAN_OPTIONS="halt_on_error=1"), timeout=300)
        raw = np.fromfile(outp, dtype=np.uint8)
        assert int(raw[:4].view(np.int32)[0]) == 0, label
        vals = raw[4:].view(np.float64)
        o = o3d.Oracle3D(w.params).init(w.rho, w.ux, w.uy, w.uz, w.T)
        o.step(steps)
        exp = np.concatenate([a.ravel() for a in o.fields()])
        print(f"[case] sanitized 3-D oracle: {label}, {steps} steps", flush=True)
        assert np.array_equal(vals[:5 * n], exp), label
