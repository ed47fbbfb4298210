"""The pins have teeth: each plausible slip, planted in a copy of the oracle
(compiled on the CPU into a temporary library), makes the pin suite fail.

Mutations: the unsquared Eq. (MSD03) update; mu instead of w*mu in the SNR;
'>=' instead of '>' in the running maximum; the sign of the anchored Eq. (sd03)
coefficient; the Eq. (MSD04) weights swapped; a shifted boxcar window; a
strict threshold; sample instead of population sigma; the MSD04 ratio
inverted; a widest-boxcar series one sample short; w instead of sqrt(w) in
Eq. (sd02); the AUTO switch at rho > kappa; and in the decimated search, the
start tested against the width instead of its stride, an inverted stride test
and a stride grid shifted by one.

The peak-finding and de-dispersion steps of the oracle (Python) get their
own slips, planted in a copy of the oracle package.  Peak-finding: '>='
instead of '>' against the neighbours, the tie broken towards the later
sample, a time radius one short, the DM radius ignored, a strict threshold.
De-dispersion: the frequency terms swapped (delays of the wrong sign),
channels counted upwards from the top frequency, delays truncated instead of
rounded, the output one sample short, the delay table read transposed, and
the dispersion constant off by the factor 1e3 of a units slip.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "spd_oracle.c")

MUTATIONS = {
    "no_square": ("S += d * d / (j * (j - 1.0));", "S += d / (j * (j - 1.0));"),
    "mu_not_wmu": ("(B - (double)W[i] * mu) / sig_w[i]", "(B - mu) / sig_w[i]"),
    "ge_ties": ("if (s > best) { best = s; bi = i; }", "if (s >= best) { best = s; bi = i; }"),
    "anchored_sign": ("coef = (sig_nmax - base) / (double)(nmax - 1);\n            flags |= FLAG_LINEAR;\n"
                      "        } else if (sigma_mode == SIG_LINEAR_LITERAL)",
                      "coef = (base - sig_nmax) / (double)(nmax - 1);\n            flags |= FLAG_LINEAR;\n"
                      "        } else if (sigma_mode == SIG_LINEAR_LITERAL)"),
    "merge_weights": ("m / (n * (m + n)) * d * d", "n / (m * (m + n)) * d * d"),
    "window_shift": ("while (k < W[i]) { B += row[t + k]; ++k; }", "while (k < W[i]) { B += row[t + k + 1]; ++k; }"),
    "threshold_strict": ("if (s >= f_T) {", "if (s > f_T) {"),
    "sample_sigma": ("double sigma = n > 0.0 ? sqrt(S / n) : 0.0;",
                     "double sigma = n > 1.0 ? sqrt(S / (n - 1.0)) : 0.0;"),
    "merge_ratio": ("double d = (n / m) * a3[1] - b3[1];", "double d = (m / n) * a3[1] - b3[1];"),
    "nmax_series_short": ("for (int k = 0; k < nmax; ++k) b += row[t + k];",
                          "for (int k = 0; k < nmax - 1; ++k) b += row[t + k];"),
    "w_not_sqrt_w": ("sig_w[i] = sqrt((double)W[i]) * sigma", "sig_w[i] = (double)W[i] * sigma"),
    "auto_at_kappa": ("if (rho > 1.0 + kappa) {", "if (rho > kappa) {"),
    "stride_by_width": ("if (stride && t % stride[i] != 0) continue;", "if (stride && t % W[i] != 0) continue;"),
    "stride_inverted": ("if (stride && t % stride[i] != 0) continue;", "if (stride && t % stride[i] == 0) continue;"),
    "stride_shifted": ("if (stride && t % stride[i] != 0) continue;", "if (stride && (t + 1) % stride[i] != 0) continue;"),
}
PINS = ["test_oracle_pins.py", "test_oracle_dit_pins.py"]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    a, b = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(a) == 1, "mutation site not found"
    c = tmp_path / ("%s.c" % name)
    c.write_text(src.replace(a, b))
    so = tmp_path / ("%s.so" % name)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(c), "-lm"])
    env = dict(os.environ, SPD_ORACLE_LIB=str(so), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"] +
                       [os.path.join(ROOT, "tests", f) for f in PINS], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, "planted mistake %s passed every pin:\n%s" % (name, r.stdout[-500:])


PY_SRC = os.path.join(ROOT, "oracle", "__init__.py")
PY_MUTATIONS = {
    "dedisp_sign": ("KDM * (1.0 / (f * f) - 1.0 / (ft * ft))", "KDM * (1.0 / (ft * ft) - 1.0 / (f * f))"),
    "dedisp_channel_up": ("f = float(f_top_mhz) - np.arange", "f = float(f_top_mhz) + np.arange"),
    "dedisp_truncate": ("np.floor(dm[:, None] * kc[None, :] + 0.5)", "np.floor(dm[:, None] * kc[None, :])"),
    "dedisp_short": ("n_out = fb.shape[1] - int(delays.max())", "n_out = fb.shape[1] - int(delays.max()) - 1"),
    "dedisp_transposed": ("k = int(delays[d, c])", "k = int(delays.T.reshape(delays.shape)[d, c])"),
    "dedisp_units": ("KDM = 4.148808e3", "KDM = 4.148808"),
    "peak_ge": ("if np.any(win > v):", "if np.any(win >= v):"),
    "peak_tie_later": ("if np.any((rr < r) | ((rr == r) & (tt < t))):", "if np.any((rr > r) | ((rr == r) & (tt > t))):"),
    "peak_t_radius_short": ("t0, t1 = max(0, t - t_radius), min(L, t + t_radius + 1)",
                            "t0, t1 = max(0, t - t_radius + 1), min(L, t + t_radius)"),
    "peak_no_dm_radius": ("r0, r1 = max(0, r - dm_radius), min(R, r + dm_radius + 1)", "r0, r1 = r, r + 1"),
    "peak_strict_threshold": ("for r, t in np.argwhere(snr >= threshold):", "for r, t in np.argwhere(snr > threshold):"),
}


@pytest.mark.parametrize("name", sorted(PY_MUTATIONS))
def test_python_pins_catch_planted_mistake(name, tmp_path):
    a, b = PY_MUTATIONS[name]
    src = open(PY_SRC).read()
    assert src.count(a) == 1, "mutation site not found"
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    (pkg / "__init__.py").write_text(src.replace(a, b))
    lib = os.path.join(ROOT, "oracle", "libspd_oracle.so")
    env = dict(os.environ, SPD_ORACLE_LIB=lib, PYTHONPATH=str(tmp_path) + os.pathsep + ROOT)
    probe = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.__file__)"], cwd=str(tmp_path),
                           env=env, capture_output=True, text=True)
    assert probe.stdout.strip().startswith(str(tmp_path)), probe.stdout + probe.stderr
    pins = "test_oracle_dedisp_pins.py" if name.startswith("dedisp") else "test_oracle_cluster_pins.py"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "--rootdir", str(tmp_path),
                        os.path.join(ROOT, "tests", pins)], cwd=str(tmp_path), env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, "planted mistake %s passed every pin:\n%s" % (name, r.stdout[-500:])
