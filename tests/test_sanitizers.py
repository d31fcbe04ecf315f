"""CPU sanitizer builds (AddressSanitizer + UndefinedBehaviorSanitizer).

1. The FP64 oracle, built with gcc -fsanitize=address,undefined, runs the
   oracle's pins: no out-of-bounds access, use after free or undefined
   behaviour on any of their paths (OpenMP loops included).
2. The library's host code (parameter checks, workspace planning, marker
   templates and patches, the overlap check), built with the sanitizers on the
   host side only (device code is not instrumented and never runs here), sizes
   every workload and rejects bad inputs; pibm_init runs its planning and
   checks and then stops at the first HIP call, since this host has no GPU.

Each runs in a subprocess with the sanitizer runtime preloaded (a sanitized
library loaded into an uninstrumented Python needs its runtime first) and
leak checking off (the interpreter itself holds memory at exit).  A
sanitizer report fails the test.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer", "SUMMARY: UndefinedBehaviorSanitizer")


def _run(cmd, env_extra, timeout):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    env.update(env_extra)
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = res.stdout + res.stderr
    bad = [r for r in REPORTS if r in out]
    assert res.returncode == 0 and not bad, out[-4000:]
    return out


@pytest.mark.slow
def test_oracle_pins_under_asan_ubsan(tmp_path):
    gcc_asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(gcc_asan):
        pytest.skip("gcc has no AddressSanitizer runtime")
    so = str(tmp_path / "libpibm_oracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                           "-o", so, os.path.join(ROOT, "oracle", "pibm_oracle.c"), "-lm"])
    # every pin except the two long steady-state runs (their code paths are
    # the same stream / collide / exchange loops the other pins cover)
    out = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_oracle_pins.py",
                "-k", "not table1_steady and not stokes_drag"],
               {"LD_PRELOAD": gcc_asan, "PIBM_ORACLE_LIB": so}, timeout=900)
    assert " passed" in out


@pytest.mark.slow
def test_library_host_planning_under_asan_ubsan(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc):
        pytest.skip("hipcc not available")
    rt = subprocess.run(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    if not os.path.exists(rt):
        pytest.skip("clang AddressSanitizer runtime not found")
    so = str(tmp_path / "libpibm_host_san.so")
    src = os.path.join(ROOT, "paper_1502_01159_amd", "csrc")
    # sanitizers on the host side only; device code unoptimised (never run here)
    subprocess.check_call([hipcc, "-O1", "-g", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
                           "-Xarch_device", "-O0", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-sanitize-recover=undefined", "-o", so,
                           os.path.join(src, "pibm.hip"), os.path.join(src, "pibm_mlp.hip")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    script = textwrap.dedent(f"""
        import ctypes, sys
        sys.path.insert(0, {ROOT!r})
        from paper_1502_01159_amd import pibm, workloads as W
        pibm.LIB_PATH = {so!r}
        L = pibm.lib()
        hip = ctypes.CDLL("libamdhip64.so")
        n = ctypes.c_int(0)
        if hip.hipGetDeviceCount(ctypes.byref(n)) == 0 and n.value > 0:
            raise SystemExit("a GPU is present: this check is for CPU-only hosts")
        for name in ["c1", "c2_small", "c3_small", "c4_small", "c2", "c3", "c4", "x3"]:
            cfg, P = W.workload(name)
            for st in ("f32", "f64", "f16", "bf16"):
                if st in ("f16", "bf16") and (cfg.get("lattice", 19) == 15 or cfg.get("thermal_model", 0) == 1):
                    continue
                p = pibm.make_params(cfg, st)
                parts = pibm.make_particles(P)
                assert L.pibm_workspace_bytes(ctypes.byref(p), parts, len(P)) > 0, (name, st)
        cfg, P = W.workload("c3_small")
        parts = pibm.make_particles(P)
        for bad in (dict(tau_f=0.5), dict(dim=4), dict(lattice=17), dict(interp_order=3), dict(streams=5)):
            p = pibm.make_params(dict(cfg, **bad))
            assert L.pibm_workspace_bytes(ctypes.byref(p), parts, len(P)) == 0, bad
        p = pibm.make_params(cfg)
        nb = L.pibm_workspace_bytes(ctypes.byref(p), parts, len(P))
        h = ctypes.c_void_p()
        fake = ctypes.c_void_p(1 << 20)          # never dereferenced: the first HIP call fails first
        assert L.pibm_init(ctypes.byref(h), ctypes.byref(p), parts, len(P), fake, nb - 1, None) == pibm.EINVAL
        assert L.pibm_init(ctypes.byref(h), ctypes.byref(p), parts, len(P), fake, nb, None) == pibm.EDEVICE
        Q = P.copy(); Q[1, :3] = Q[0, :3]        # two centres on top of each other
        assert L.pibm_init(ctypes.byref(h), ctypes.byref(p), pibm.make_particles(Q), len(Q), fake, nb,
                           None) == pibm.EOVERLAP
        Q = P.copy(); Q[0, 0] = -50.0            # outside the walls
        assert L.pibm_init(ctypes.byref(h), ctypes.byref(p), pibm.make_particles(Q), len(Q), fake, nb,
                           None) == pibm.EINVAL
        for k in range(-8, 2):
            L.pibm_strerror(k)
        assert L.pibm_mlp_workspace_bytes(4096) > 0 and L.pibm_mlp_workspace_bytes(0) == 0
        print("host planning ok")
    """)
    out = _run([sys.executable, "-c", script], {"LD_PRELOAD": rt}, timeout=600)
    assert "host planning ok" in out
