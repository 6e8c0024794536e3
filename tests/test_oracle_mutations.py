"""The oracle's pins catch plausible mistakes (CPU).

Each case plants one mistake in a temporary copy of `oracle/` (a dropped term, a wrong
sign, index or coefficient, a transposed operand) and runs the oracle pin tests against
that copy in a subprocess; the case passes when at least one pin fails. The repository's
own oracle is never modified.

Mistakes that cannot change any result are not listed: exchanging cos and sin in a
chart is a reflection of the plane, which leaves every distance (and so every kernel
matrix) unchanged.
"""

import concurrent.futures
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["test_oracle_pins.py", "test_oracle_cf.py", "test_oracle_chart3d.py", "test_oracle_hypergrad.py",
             "test_oracle_mgvi.py"]

ICR = "icr_oracle.py"
CF = "cf_oracle.py"

# (file, text as written, planted mistake, what it breaks)
MUTATIONS = [
    (ICR, "k = (1.0 + a + a * a / 3.0) * np.exp(-a)", "k = (1.0 + a + a * a / 2.0) * np.exp(-a)",
     "Matern-5/2 quadratic coefficient"),
    (ICR, "        a = math.sqrt(3.0) * t\n        k = (1.0 + a) * np.exp(-a)",
     "        a = math.sqrt(2.0) * t\n        k = (1.0 + a) * np.exp(-a)", "Matern-3/2 scaling"),
    (ICR, "k = np.exp(-0.5 * t * t)", "k = np.exp(-t * t)", "squared-exponential exponent"),
    (ICR, "shapes.append(tuple(2 * (n - 2) for n in prev))", "shapes.append(tuple(2 * (n - 1) for n in prev))",
     "level size recursion"),
    (ICR, "org.append(org[-1] + 0.75 * spac[l])", "org.append(org[-1] + 0.5 * spac[l])", "level origin"),
    (ICR, "return (wins * dl)[None], ((kids - 0.5) * dl / 2.0)[None]",
     "return (wins * dl)[None], ((kids - 0.5) * dl / 4.0)[None]", "child offset delta/4 -> delta/8"),
    (ICR, "kid_idx = centre[:, None, :] + (kids[None] - 0.5) * dl / 2.0",
     "kid_idx = centre[:, None, :] + (kids[None] - 0.5) * dl", "charted child offset"),
    (ICR, "itertools.product((-1, 0, 1), repeat=ndim)", "itertools.product((-1, 0, 2), repeat=ndim)",
     "window offsets"),
    (ICR, "root = np.sqrt(np.where(bad, 1.0, piv))", "root = np.where(bad, 1.0, piv)", "Cholesky pivot root"),
    (ICR, "bad = ~(piv > tau)", "bad = ~(piv > 10.0 * tau)", "clamp threshold"),
    (ICR, "d_mat = k_ff - r_mat @ np.swapaxes(k_fc, -1, -2)", "d_mat = k_ff + r_mat @ np.swapaxes(k_fc, -1, -2)",
     "sign of the conditional covariance update"),
    (ICR, "window = s[lead + tuple(slice(1 + w[a], nc[a] - 1 + w[a]) for a in range(ndim))]",
     "window = s[lead + tuple(slice(1 - w[a], nc[a] - 1 - w[a]) for a in range(ndim))]",
     "mirrored window in the forward"),
    (ICR, "acc = acc + _coef(sqrt_d, ib, jb) * fresh", "acc = acc + _coef(sqrt_d, jb, ib) * fresh",
     "transposed sqrt(D) in the forward"),
    (ICR, "acc = sum(_coef(sqrt_d, ib, jb) * blocks[ib] for ib in range(len(kids)))",
     "acc = sum(_coef(sqrt_d, jb, ib) * blocks[ib] for ib in range(len(kids)))",
     "untransposed sqrt(D) in the adjoint"),
    (ICR, "acc = sum(_coef(r_mat, ib, iw) * blocks[ib] for ib in range(len(kids)))",
     "acc = sum(_coef(r_mat, ib, len(wins) - 1 - iw) * blocks[ib] for ib in range(len(kids)))",
     "wrong window index in the adjoint"),
    (ICR, "s = (xi[..., self.level_slice(0)] @ self.l00.T)", "s = (xi[..., self.level_slice(0)] @ self.l00)",
     "transposed L00 in the forward"),
    (ICR, "out[..., self.level_slice(0)] = y.reshape(batch + (-1,)) @ self.l00",
     "out[..., self.level_slice(0)] = y.reshape(batch + (-1,)) @ self.l00.T", "transposed L00 in the adjoint"),
    (ICR, "return self.adjoint(np.asarray(w, dtype=np.float64) * self.forward(v)) + v",
     "return self.adjoint(np.asarray(w, dtype=np.float64) * self.forward(v))", "dropped +v of the metric"),
    (ICR, "dk = a * a * (1.0 + a) / 3.0 * np.exp(-a)", "dk = a * a * (1.0 + a) / 2.0 * np.exp(-a)",
     "Matern-5/2 length derivative"),
    (ICR, "phi = np.tril(x) - 0.5 * np.eye(n)", "phi = np.tril(x) - 0.25 * np.eye(n)",
     "halved diagonal of the Cholesky derivative"),
    (ICR, "d_d = dk_ff - d_r @ np.swapaxes(k_fc, -1, -2) - r_mat @ np.swapaxes(dk_fc, -1, -2)",
     "d_d = dk_ff - d_r @ np.swapaxes(k_fc, -1, -2)", "dropped term of dD"),
    (ICR, "g_sigma = np.sum(ybar * s_final, axis=-1) / model.cfg.scale",
     "g_sigma = np.sum(ybar * s_final, axis=-1) * model.cfg.scale", "scale gradient"),
    (ICR, "p = r + (rr_new / rr) * p\n        rr = rr_new\n    return x",
     "p = r + (rr / rr_new) * p\n        rr = rr_new\n    return x", "CG direction update"),
    (ICR, "p = r + (rr_new / rr) * p\n        rr = rr_new\n        new_energy",
     "p = r + (rr / rr_new) * p\n        rr = rr_new\n        new_energy", "CG direction update of the SL rule"),
    (ICR, "return 0.5 * float(x @ mx) - float(b @ x)", "return 0.5 * float(x @ mx) + float(b @ x)",
     "sign of the CG energy"),
    (ICR, "if decreases[-1] < absdelta:", "if decreases[-1] > absdelta:", "energy stopping rule"),
    (ICR, "r = weighted_adjoint(model, w, 0.5, eta_data, add=eta_xi)",
     "r = weighted_adjoint(model, w, 1.0, eta_data, add=eta_xi)", "sample noise weight power"),
    (ICR, "r = r0 * np.exp(g * points[..., 0])\n    th = a * points[..., 1]\n    return np.stack([r * np.cos(th), r * np.sin(th)], axis=-1)",
     "r = r0 * np.exp(g * points[..., 1])\n    th = a * points[..., 1]\n    return np.stack([r * np.cos(th), r * np.sin(th)], axis=-1)",
     "log-radial chart radius axis"),
    (CF, "return f.real - f.imag", "return f.real + f.imag", "Hartley sign"),
    (CF, "return hartley2(x) / np.sqrt(x.shape[-2] * x.shape[-1])",
     "return hartley2(x) / (x.shape[-2] * x.shape[-1])", "transform normalisation"),
    (CF, "** (-slope / 4.0)", "** (-slope / 2.0)", "amplitude exponent"),
    (CF, "k = np.minimum(np.arange(n), n - np.arange(n)).astype(np.float64)",
     "k = np.arange(n).astype(np.float64)", "harmonic numbers not folded"),
    (CF, "return v + amp * transform(lam * transform(amp * v))", "return v + amp * transform(lam * transform(v))",
     "dropped amplitude in M_p"),
]


def _mutated_tree(base, fname, old, new):
    dst = base / "tree"
    shutil.copytree(os.path.join(ROOT, "oracle"), dst / "oracle",
                    ignore=shutil.ignore_patterns("__pycache__", "*.so", "*.o"))
    shutil.copytree(os.path.join(ROOT, "tests"), dst / "tests", ignore=shutil.ignore_patterns("__pycache__"))
    for extra in ("workloads.py", "pytest.ini"):
        shutil.copy(os.path.join(ROOT, extra), dst / extra)
    path = dst / "oracle" / fname
    text = path.read_text()
    assert text.count(old) == 1, f"the text to mutate must appear once in {fname}: {old!r}"
    path.write_text(text.replace(old, new))
    return dst


def _run_pins(tree):
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           *[os.path.join("tests", f) for f in PIN_FILES]]
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1", OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1")
    return subprocess.run(cmd, cwd=tree, capture_output=True, text=True, env=env, timeout=600)


@pytest.fixture(scope="module")
def pin_runs(tmp_path_factory):
    """Return code and output of the pins on the unmutated copy (key None) and on every
    mutation, run as concurrent subprocesses."""
    cases = [(None, (CF, "return f.real - f.imag", "return f.real - f.imag"))]
    cases += [(m[3], m[:3]) for m in MUTATIONS]

    trees = [(key, _mutated_tree(tmp_path_factory.mktemp("mutant"), *m)) for key, m in cases]

    def run(case):
        key, tree = case
        r = _run_pins(tree)
        return key, (r.returncode, r.stdout[-2000:] + r.stderr[-2000:])

    workers = max(1, min(8, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        return dict(pool.map(run, trees))


def test_unmutated_copy_passes_the_pins(pin_runs):
    code, out = pin_runs[None]
    assert code == 0, out


@pytest.mark.parametrize("what", [m[3] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(pin_runs, what):
    code, out = pin_runs[what]
    assert code == 1, f"{what}: no pin failed\n" + out
