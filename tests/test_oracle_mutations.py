"""Planted mistakes in the oracle must each fail at least one CPU pin.

Each case copies ``oracle/`` and the oracle's pin tests into a temporary
directory, plants one plausible mistake in the copy (a dropped factor, a
wrong sign, index or power, a transposed or conjugated operand), and runs
the pin tests there.  The case passes when that run fails.  The repository's
own oracle is never modified.

The cases cover the parts the paper defines (Sec. II-A basis and expansion,
Eq. (2) score and gradient, Sec. II-C ascent and Newton refinement, the
energy ratio of the Fig. 1 caption) and the readings the oracle takes where
the paper is silent (step weight, natural gradient, Euler wrap).
"""

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PIN_TESTS = ["test_oracle_basis.py", "test_oracle_wigner.py", "test_oracle_score.py",
             "test_oracle_align.py", "test_oracle_refine.py", "test_oracle_scale.py",
             "test_oracle_shift.py", "test_fold_identity.py", "test_paper_parameters.py"]

# (name, file under oracle/, text, replacement)
MUTATIONS = [
    ("expansion cell volume h^2", "expand.py",
     "(h ** 3) * (F @ basis_conj)", "(h ** 2) * (F @ basis_conj)"),
    ("expansion without conj", "expand.py",
     "basis_conj = np.conj(rad[:, None] * Y)", "basis_conj = rad[:, None] * Y"),
    ("expansion m order reversed", "expand.py",
     "Yall[l][np.arange(-l, l + 1)].T", "Yall[l][np.arange(l, -l - 1, -1)].T"),
    ("normalisation sqrt(3)", "basis.py",
     "np.sqrt(2.0) / abs(special.spherical_jn(l + 1, lam))",
     "np.sqrt(3.0) / abs(special.spherical_jn(l + 1, lam))"),
    ("band cut-off at lambda_{L,1}", "basis.py",
     "return first_zero(L + 1)", "return first_zero(L)"),
    ("step weight l^2", "score.py",
     "np.sum(ll * (ll + 1) * na * nb)", "np.sum(ll * ll * na * nb)"),
    ("step weight over all k", "score.py",
     "sel = keep & (idx.l == l)", "sel = idx.l == l"),
    ("cross-power conjugated", "score.py",
     "np.outer(np.conj(bl), al)", "np.outer(bl, np.conj(al))"),
    ("cross-power transposed", "score.py",
     "np.outer(np.conj(bl), al)", "np.outer(np.conj(bl), al).T"),
    ("gradient alpha uses n", "score.py",
     "G[:, 0] += np.real(np.sum(W * d * (-1j * m)[None, :, None], axis=(1, 2)))",
     "G[:, 0] += np.real(np.sum(W * d * (-1j * m)[None, None, :], axis=(1, 2)))"),
    ("gradient beta sign", "score.py",
     "G[:, 1] += np.real(np.sum(W * dp, axis=(1, 2)))",
     "G[:, 1] -= np.real(np.sum(W * dp, axis=(1, 2)))"),
    ("Hessian alpha-gamma uses alpha twice", "score.py",
     "H[:, 0, 2] += re(W * d * fa * fg)", "H[:, 0, 2] += re(W * d * fa * fa)"),
    ("energy ratio off by one degree", "score.py",
     "tail = tot - np.cumsum(E)", "tail = tot - np.cumsum(E) + E"),
    ("band selection strict", "score.py",
     "hit = np.nonzero(r <= tau)[0]", "hit = np.nonzero(r < tau)[0]"),
    ("batch band at the upper half", "score.py",
     "need = (B + 1) // 2", "need = B // 2"),
    ("D with +i m alpha", "wigner.py",
     "np.exp(-1j * m * alpha)[:, None]", "np.exp(1j * m * alpha)[:, None]"),
    ("J_y sign", "wigner.py",
     "jy = (jp - jp.T) / 2j", "jy = (jp.T - jp) / 2j"),
    ("d' sign", "wigner.py",
     "np.matmul(-1j * jy, d)", "np.matmul(1j * jy, d)"),
    ("Euler wrap keeps alpha", "wigner.py",
     "        a += np.pi\n", "        a += 0.0\n"),
    ("natural gradient sign of the metric term", "align.py",
     "da = (G[:, 0] - c * G[:, 2]) / s2", "da = (G[:, 0] + c * G[:, 2]) / s2"),
    ("Newton step sign", "align.py",
     "d[i] = np.linalg.solve(Hn, G[i])", "d[i] = -np.linalg.solve(Hn, G[i])"),
    ("shift direction", "expand.py",
     "out[dst[0], dst[1], dst[2]] = f[src[0], src[1], src[2]]",
     "out[src[0], src[1], src[2]] = f[dst[0], dst[1], dst[2]]"),
]


def _run_mutant(case):
    name, fname, old, new = case
    with tempfile.TemporaryDirectory(prefix="oracle_mut_") as tmp:
        shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(tmp, "oracle"),
                        ignore=shutil.ignore_patterns("__pycache__"))
        shutil.copytree(os.path.join(ROOT, "synth"), os.path.join(tmp, "synth"),
                        ignore=shutil.ignore_patterns("__pycache__"))
        os.makedirs(os.path.join(tmp, "tests"))
        for f in ["conftest.py", *PIN_TESTS]:
            shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(tmp, "tests", f))
        shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(tmp, "tests", "golden"))
        shutil.copy(os.path.join(ROOT, "pytest.ini"), os.path.join(tmp, "pytest.ini"))
        path = os.path.join(tmp, "oracle", fname)
        src = open(path).read()
        if src.count(old) != 1:
            return name, "stale", f"text occurs {src.count(old)} times in {fname}"
        open(path, "w").write(src.replace(old, new))
        env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1", OMP_NUM_THREADS="1",
                   OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            "-m", "not gpu", *[os.path.join("tests", t) for t in PIN_TESTS]],
                           cwd=tmp, env=env, capture_output=True, text=True, timeout=600)
        if r.returncode == 1:
            return name, "killed", ""
        return name, "survived" if r.returncode == 0 else f"rc={r.returncode}", r.stdout[-2000:]


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin():
    workers = max(1, min(8, (os.cpu_count() or 2) // 2))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(_run_mutant, MUTATIONS))
    bad = [(n, s, out) for n, s, out in results if s != "killed"]
    assert not bad, "\n".join(f"{n}: {s}\n{out}" for n, s, out in bad)
