"""Mutation audit of the oracle's pins (a development check, not collected
by pytest; CPU only, about ten minutes with four workers).

Each mutant is a temporary copy of the repository with ONE planted mistake
in oracle/ (a wrong sign, factor, index, level or dropped term); the pins of
the oracle (tests/test_oracle_*.py, which compare it with what the paper and
the mathematics fix, never with the library) must fail on every one.

    python tests/mutation_audit.py            # all mutants
    python tests/mutation_audit.py 3 12       # selected ones
"""
import glob
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# (file, original text, planted mistake, what it breaks)
L, H, Q, A = "oracle/lbm.py", "oracle/hostmap.py", "oracle/measure.py", "oracle/adjoint.py"
MUTS = [
 (L, "1 / 12, 1 / 12, 1 / 12, 1 / 12])", "1 / 12, 1 / 12, 1 / 12, 1 / 6])", "stencil diagonal weight"),
 (L, "phi = (1.0 + v + v * v - v ** 3)", "phi = (1.0 + v + v * v + v ** 3)", "CS phi sign"),
 (L, "- 4.0 * v ** 3 + v ** 4) / one_m ** 4", "+ 4.0 * v ** 3 + v ** 4) / one_m ** 4", "CS dphi sign"),
 (L, "p_lbe = p_eos + 0.5 * co.G2 * rho * rho", "p_lbe = p_eos + co.G2 * rho * rho", "p_LBE G2 term"),
 (L, "dp_lbe = dp_eos + co.G2 * rho", "dp_lbe = dp_eos + 0.5 * co.G2 * rho", "dp_LBE G2 term"),
 (L, "2.0 * ALPHA1 * rho + 2.0 * BETA1 * eta + 3.0 * rho * u2,", "2.0 * ALPHA1 * rho + 2.0 * BETA1 * eta + 2.0 * rho * u2,", "meq e u2"),
 (L, "- 3.0 * rho * u2 + 9.0 * rho * ux * ux * uy * uy,", "- 3.0 * rho * u2 + 6.0 * rho * ux * ux * uy * uy,", "meq eps quartic"),
 (L, "-rho * ux + 3.0 * rho * ux * uy * uy,", "-rho * ux + 3.0 * rho * ux * ux * uy,", "meq q_x cubic"),
 (L, "co.alpha2 * rho + co.beta2 * eta", "co.alpha2 * rho - co.beta2 * eta", "meq eps eta sign"),
 (L, "-6.0 * Fu + 9.0 * (2.0 * Fx * ux * uy * uy", "-6.0 * Fu + 9.0 * (1.0 * Fx * ux * uy * uy", "F_m eps"),
 (L, "-Fx + 3.0 * (Fx * uy * uy + 2.0 * Fy * ux * uy)", "-Fx + 3.0 * (Fx * uy * uy + Fy * ux * uy)", "F_m q_x"),
 (L, "2.0 * (Fx * ux - Fy * uy),", "(Fx * ux - Fy * uy),", "F_m p_xx"),
 (L, "zero, 0.5 * q, -0.5 * q, zero", "zero, 0.5 * q, 0.5 * q, zero", "Q_m eps sign"),
 (L, "(Ftx * Ftx - Fty * Fty) / 12.0", "(Ftx * Ftx - Fty * Fty) / 6.0", "Q_m p_xx"),
 (L, "Ftx * Fty / 12.0])", "Ftx * Fty / 6.0])", "Q_m p_xy"),
 (L, "S[1, 2] = co.k * co.s_eps * we", "S[1, 2] = co.k * co.s_eps * wp", "S_12 factor"),
 (L, "S[7, 6] = -2.0 * co.bs * uy", "S[7, 6] = 2.0 * co.bs * uy", "S_76 sign"),
 (L, "S[8, 4] = co.bs * uy * co.s_q * wp", "S[8, 4] = co.bs * ux * co.s_q * wp", "S_84 index"),
 (L, "S[1, 4] = co.h * ux * co.s_q * we", "S[1, 4] = co.h * uy * co.s_q * we", "S_14 index"),
 (L, "jx = np.tensordot(CX.astype(float), f, axes=(0, 0)) + 0.5 * Fx", "jx = np.tensordot(CX.astype(float), f, axes=(0, 0)) + 1.0 * Fx", "half force in u"),
 (L, "Ftx=G * gx", "Ftx=co.G2 * gx", "F-tilde scale"),
 (L, "- _mv(R, _mv(I - 0.5 * S, d))", "- _mv(R, d)", "R acts on (I - S/2) d"),
 (L, "_mv(S, Qm)", "Qm", "S Q_m"),
 (L, "co.k * (0.5 * co.s_e - 1.0) * co.s_eps * Qm[2]", "0.0 * Qm[2]", "seq step 6 coupling"),
 (L, "0.5 * co.h * co.s_q * (ux * m[4] + uy * m[6])", "co.h * co.s_q * (ux * m[4] + uy * m[6])", "seq step 2 h"),
 (L, "shift=(CY[i], CX[i])", "shift=(CX[i], CY[i])", "stream axes"),
 (L, "R[1, 8] = (12.0 * sp", "R[1, 8] = (6.0 * sp", "R_18 factor"),
 (L, "X[7, 1] = -3.0 * (2.0 - sp) * b * (-ux2 * uy)", "X[7, 1] = -3.0 * (2.0 - sp) * b * (ux2 * uy)", "X_71 sign"),
 (L, "return np.array([1.0, co.s_e, co.s_eps, 1.0, co.s_q, 1.0, co.s_q, co.s_p, co.s_p])", "return np.array([1.0, co.s_e, co.s_eps, 1.0, co.s_q, 1.0, co.s_q, co.s_p, co.s_e])", "rate of p_xy"),
 (L, "eta = (3.0 * p_lbe - (2.0 + ALPHA1) * rho) / BETA1", "eta = (3.0 * p_lbe - (2.0 - ALPHA1) * rho) / BETA1", "eta from p_LBE"),
 (H, "h = 6.0 * varpi * (1.0 - varpi) / (1.0 - 3.0 * varpi)", "h = 6.0 * varpi / (1.0 - 3.0 * varpi)", "h of Eq. 7"),
 (H, "bs = (1.0 - varpi) / (1.0 - 3.0 * varpi)", "bs = (1.0 + varpi) / (1.0 - 3.0 * varpi)", "b of Eq. 7"),
 (H, "beta2 = -2.0 * beta1 / (1.0 - varpi)", "beta2 = -2.0 * beta1 / (1.0 + varpi)", "beta2"),
 (H, "tau_e = 1.0 / (12.0 * (k + 1.0) * tau_q)", "tau_e = 1.0 / (12.0 * k * tau_q)", "tau_e"),
 (H, "kappa = a / 2.0", "kappa = a / 4.0", "kappa"),
 (H, "r5 = 0.95 * rg + 0.05 * rl", "r5 = 0.9 * rg + 0.1 * rl", "thickness levels"),
 (H, "k_eos = sigma / (c_sigma * k_int)", "k_eos = sigma / c_sigma", "K_EOS map"),
 (H, "return c_sigma / (3.0 * k_int * cs_repulsive_slope(rl, rt, b))", "return c_sigma / (3.0 * k_int * cs_repulsive_slope(0.9 * rl, rt, b))", "sigma_paper at rho_l"),
 (Q, "lo = level_crossings(profile, 0.95 * rho_g + 0.05 * rho_l)", "lo = level_crossings(profile, 0.9 * rho_g + 0.1 * rho_l)", "measure: width level"),
 (Q, "level = 0.5 * (rho_g + rho_l)", "level = 0.5 * rho_l", "measure: radius level"),
 (Q, "return float(2 * np.pi * s.sum() / (k * s).sum())", "return float(np.pi * s.sum() / (k * s).sum())", "measure: domain length"),
 (Q, "return float((p_in - p_out) * R), R, float(p_in - p_out)", "return float((p_in - p_out) * R * 0.5), R, float(p_in - p_out)", "measure: laplace 2D"),
 (A, "for dy in range(-2, 3):", "for dy in range(-1, 2):", "adjoint: influence box"),
 (A, "g = (lam0 * drho).sum(axis=0) / H", "g = (lam0 * drho[::-1]).sum(axis=0) / H", "adjoint: equilibrium order"),
 (A, "return ((r - target) ** 2).sum()", "return (np.abs(r - target) ** 2).sum()", "adjoint: loss not analytic"),
 (Q, "np.sort(np.concatenate([on, idx + a[idx] / (a[idx] - b[idx])]))", "np.sort(np.concatenate([on, idx + b[idx] / (a[idx] - b[idx])]))", "measure: interpolation"),
]


def run(j, base):
    """Mutant j (j < 0: the unmutated control, which must pass)."""
    path, old, new, name = MUTS[j] if j >= 0 else (MUTS[0][0], "", "", "control (no mutation)")
    d = os.path.join(base, f"m{j:02d}" if j >= 0 else "control")
    # the oracle's pins need only the oracle, the input generators and the tests
    for sub in ("oracle", "workloads", "tests"):
        shutil.copytree(os.path.join(ROOT, sub), os.path.join(d, sub),
                        ignore=shutil.ignore_patterns("__pycache__", ".pytest_cache"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), d)
    if j >= 0:
        src = open(os.path.join(d, path)).read()
        if src.count(old) != 1:
            return j, name, "NO-MATCH", ""
        with open(os.path.join(d, path), "w") as fh:
            fh.write(src.replace(old, new))
    pins = sorted(glob.glob(os.path.join(d, "tests", "test_oracle_*.py")))
    r = subprocess.run([sys.executable, "-m", "pytest", *pins, "-x", "-q", "-p", "no:cacheprovider"],
                       cwd=d, capture_output=True, text=True)
    lines = r.stdout.strip().splitlines()
    first = next((l for l in lines if l.startswith(("FAILED", "ERROR"))), lines[-1] if lines else "")
    shutil.rmtree(d, ignore_errors=True)
    return j, name, "caught" if r.returncode != 0 else "SURVIVED", first


def main(argv):
    sel = [int(a) for a in argv] or list(range(len(MUTS)))
    with tempfile.TemporaryDirectory() as base, ThreadPoolExecutor(4) as ex:
        control = run(-1, base)
        if control[2] != "SURVIVED":  # the unmutated copy must pass its pins
            print("control run failed:", control[3])
            return 1
        print("control (no mutation): pins pass")
        res = list(ex.map(lambda j: run(j, base), sel))
    for j, name, status, first in res:
        print(f"{j:2d} {status:9s} {name:28s} {first[:110]}")
    bad = [r for r in res if r[2] != "caught"]
    print(f"{len(res) - len(bad)} of {len(res)} mutants caught")
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
