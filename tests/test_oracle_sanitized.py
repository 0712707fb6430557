"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a copy of
oracle.c built with -fsanitize=address,undefined runs small networks of both
reproducible modes (stimulus, consolidation, wrap-around grids) in a child
process; it must report nothing and give the same rasters and synapses as the
normal build."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if p.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_clean_under_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    so = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-fsanitize=address,undefined",
                           "-fno-omit-frame-pointer", "-o", str(so),
                           os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    script = textwrap.dedent(f"""
        import sys, numpy as np
        sys.path.insert(0, {ROOT!r})
        from oracle import oracle as O
        from paper_1310_8478_amd import workloads as W
        out = []
        for mode in (W.SUM_FIXED, W.SUM_ORDERED):
            cfg = W.make_config(grid_x=3, grid_y=2, neurons_per_column=70, synapses_per_neuron=25,
                                thalamic_rate=2.5, w_exc_init=9.0, weight_update_period=40,
                                sum_mode=mode, seed=77)
            n = O.Net(cfg, 130)
            n.set_stimulus(*W.stimulus_list(420, 120, 50, seed=3))
            n.run(130)
            tt, ii = n.raster()
            s = n.synapses()
            n.close()
            out.append(int(len(tt)))
            out.append(int(tt.astype(np.int64).sum() + 3 * ii.astype(np.int64).sum()))
            out.append(s["w"].tobytes().hex()[:64] + s["P"].tobytes().hex()[-64:])
        print("RESULT", out)
    """)
    env = dict(os.environ, DPSNN_ORACLE_LIB=str(so), LD_PRELOAD=f"{asan} {ubsan}",
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, env=env,
                       timeout=600)
    report = p.stdout + p.stderr
    assert p.returncode == 0, report[-3000:]
    assert "runtime error" not in report and "AddressSanitizer" not in report, report[-3000:]
    san = [line for line in p.stdout.splitlines() if line.startswith("RESULT")]
    env_plain = {k: v for k, v in os.environ.items() if k not in ("DPSNN_ORACLE_LIB",)}
    q = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True,
                       env=env_plain, timeout=600)
    assert q.returncode == 0, q.stderr[-3000:]
    plain = [line for line in q.stdout.splitlines() if line.startswith("RESULT")]
    assert san == plain and san, (san, plain)
