"""Plant one plausible mistake at a time in a scratch copy of the oracle (CPU
only) and check that the pins in test_oracle_pins.py catch every one of them.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = [
    # (file, original, mutated)  -- dropped/wrong-signed terms, transposes
    ("svgp.py", "+ np.trace(Kt @ T) - M", "+ np.trace(Kt @ T) + M"),
    ("svgp.py", "P = 2.0 * T - T @ Kt @ T", "P = 2.0 * T - Kt @ T @ T"),
    ("svgp.py", "- logdetT - np.sum(np.log(s)))", "- logdetT + np.sum(np.log(s)))"),
    ("svgp.py", "+ m @ P @ Kuu @ P @ m", "+ m @ Kuu @ P @ m"),
    ("svgp.py", "X = np.tril(W) - 0.5", "X = np.tril(W, -1) - 0.5"),
    ("svgp.py", '"fro") / np.sqrt(M)', '"fro")'),
    ("svgp.py", '"fro") / np.sqrt(M)', '"fro") / M'),
    ("svgp.py", "return L @ X", "return X @ L"),
    ("svgp.py", "G_Kt = -T @ G_P @ T - 0.5 * T", "G_Kt = -T @ G_P @ T + 0.5 * T"),
    ("svgp.py", "g_m = P @ Ka - P @ KPm", "g_m = P @ Ka - Kuu @ KPm"),
    ("svgp.py", "data = (N / B) * np.sum(E)", "data = np.sum(E)"),
    ("svgp.py", "g_Z[:, d] = -(np.sum((Huu + Huu.T) * dzz, axis=1)",
     "g_Z[:, d] = -(np.sum(Huu * dzz, axis=1)"),
    ("svgp.py", "P = 2.0 * T - T @ (Kt @ T)", "P = T - T @ (Kt @ T)"),
    ("svgp.py", "mu = Kus.T @ (P @ m)", "mu = Kus.T @ (T @ m)"),
    ("svgp.py", "var = sf2 - np.sum(Kus * (P @ Kus), axis=0)", "var = sf2 - np.sum(Kus * (T @ Kus), axis=0)"),
    ("svgp.py", "vy = var + float(noise_var)", "vy = var"),
    ("svgp.py", "lpd = log_ndtr(y * mu / np.sqrt(1.0 + var))", "lpd = log_ndtr(y * mu / np.sqrt(var))"),
    ("svgp.py", "R = Kuf - A @ (T @ Kuf)", "R = Kuf - T @ (A @ Kuf)"),
    ("svgp.py", "return float(np.sum(R * R)) / float(sigma2)", "return float(np.sum(R * R))"),
    ("svgp.py", "thr = 2.0 * float(noise_obs) * float(eps)", "thr = float(noise_obs) * float(eps)"),
    ("svgp.py", "trPK = 2.0 * trWu - trWWu", "trPK = trWu - trWWu"),
    ("svgp.py", "trWWu = np.sum(WO * WuO) / K", "trWWu = np.sum(WO * WO) / K"),
    ("svgp.py", "P = T @ (2.0 * np.eye(M) - Kt @ T)", "P = T @ (2.0 * np.eye(M) - Kuu @ T)"),
    ("svgp.py", "G_Kuu = TO - 0.25 * (A2 + A2.T)", "G_Kuu = TO + 0.25 * (A2 + A2.T)"),
    ("svgp.py", "A1 = T @ Kuu @ TO ", "A1 = T @ T @ TO "),
    ("svgp.py", "- 0.25 * (A1 + A1.T) - 0.5 * TO", "- 0.25 * (A1 + A1.T) + 0.5 * TO"),
    ("svgp.py", 'out["m"] = np.stack([g["m"] for g in gs])', 'out["m"] = np.stack([g["m"] for g in gs[::-1]])'),
    ("svgp.py", 'KL=sum(p["KL"] for p in parts)', 'KL=parts[0]["KL"]'),
    ("svgp.py", "parts = [rsvgp_bound(X, Y[:, q], N", "parts = [rsvgp_bound(X, Y[:, 0], N"),
    ("quadrature.py", "* y / np.sqrt(2.0 * v)", "* y / np.sqrt(v)"),
    ("quadrature.py", "np.exp(log_phi - log_ndtr(z))", "np.exp(log_phi + log_ndtr(z))"),
    ("quadrature.py", "E = -0.5 * LOG_2PI - 0.5 * np.log(s2) - (r * r + v) / (2.0 * s2)",
     "E = -0.5 * LOG_2PI - 0.5 * np.log(s2) - (r * r - v) / (2.0 * s2)"),
]


@pytest.mark.parametrize("fname,orig,mut", MUTATIONS, ids=[m[2][:40] for m in MUTATIONS])
def test_planted_oracle_mistake_is_caught(tmp_path, fname, orig, mut):
    dst = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "oracle"), dst / "oracle")
    shutil.copytree(os.path.join(ROOT, "tests"), dst / "tests",
                    ignore=shutil.ignore_patterns("__pycache__", "test_oracle_mutations.py"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), dst / "pytest.ini")
    path = dst / "oracle" / fname
    src = path.read_text()
    assert src.count(orig) == 1, f"mutation anchor not found once: {orig!r}"
    path.write_text(src.replace(orig, mut))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q",
                        "tests/test_oracle_pins.py"], cwd=dst,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch: {mut!r}\n{r.stdout[-500:]}"
