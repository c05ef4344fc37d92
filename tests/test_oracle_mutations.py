"""Planted mistakes in the oracle must each fail at least one pin.

Each mutant is a one-site textual change of ``oracle/rotvote_oracle.c`` of the
kind a careful reader could still make (a dropped term, a flipped sign, a wrong
index, a transposed operand, an off-by-one).  The mutant is compiled into a
temporary directory and the pins run in a child process, so a mutant that
crashes counts as caught without taking the test runner down.
"""
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

import pytest

import oracle

ROOT = Path(__file__).resolve().parents[1]

MUTANTS = [
    ("table half-step dropped", "(double)(2 * j + 1 - J)", "(double)(2 * j - J)"),
    ("cos/sin swapped", "C[j] = (float)cos(th);", "C[j] = (float)sin(th);"),
    ("residual bound halved", "return (float)(4.0 * s * s);", "return (float)(2.0 * s * s);"),
    ("norm uses wrong component", "s = s + v[2] * v[2];", "s = s + v[1] * v[2];"),
    ("dot product sign", "d = d + a[2] * b[2];", "d = d - a[2] * b[2];"),
    ("cross product transposed", "c[0] = a[1] * b[2] - a[2] * b[1];",
     "c[0] = a[2] * b[1] - a[1] * b[2];"),
    ("diagonal of M sign", "g[m + 1] = 2.0f * (a[m] * b[m]) - d;",
     "g[m + 1] = 2.0f * (a[m] * b[m]) + d;"),
    ("argmax flipped", "if (g[k] > g[ks])", "if (g[k] < g[ks])"),
    ("first column diagonal", "up[0] = 1.0f + g[0];", "up[0] = 1.0f - g[0];"),
    ("off-diagonal of M", "up[n + 1] = a[n] * b[m] + a[m] * b[n];",
     "up[n + 1] = a[n] * b[m] - a[m] * b[n];"),
    ("column w entry sign", "up[0] = c[m];", "up[0] = -c[m];"),
    ("column diagonal entry", "up[n + 1] = 1.0f + g[ks];", "up[n + 1] = 1.0f - g[ks];"),
    ("second basis w sign", "v[0] = -bu;", "v[0] = bu;"),
    ("second basis cross order", "v[1] = u[0] * b[0] + (b[1] * u[3] - b[2] * u[2]);",
     "v[1] = u[0] * b[0] + (b[2] * u[2] - b[1] * u[3]);"),
    ("second basis index", "v[3] = u[0] * b[2] + (b[0] * u[2] - b[1] * u[1]);",
     "v[3] = u[0] * b[1] + (b[0] * u[2] - b[1] * u[1]);"),
    ("basis normalisation dropped term", "r2 = r2 + up[3] * up[3];", "r2 = r2 + up[2] * up[3];"),
    ("canonical sign flipped", "neg = q[0] < 0.0f;", "neg = q[0] > 0.0f;"),
    ("equator tie-break dropped", "neg = q[1] < 0.0f;", "neg = 0;"),
    ("chart pole", "float den = 1.0f + qc[0];", "float den = 1.0f - qc[0];"),
    ("chart component shift", "t[c] = fmaf(qc[c + 1], rh, h);", "t[c] = fmaf(qc[c], rh, h);"),
    ("chart offset dropped", "t[c] = fmaf(qc[c + 1], rh, h);", "t[c] = qc[c + 1] * rh;"),
    ("grid layout transposed", "return (ic[2] * G + ic[1]) * G + ic[0];",
     "return (ic[0] * G + ic[1]) * G + ic[2];"),
    ("sample weights swapped", "q[c] = fmaf(Cj, u[c], Sj * v[c]);",
     "q[c] = fmaf(Sj, u[c], Cj * v[c]);"),
    ("sample drops second basis", "q[c] = fmaf(Cj, u[c], Sj * v[c]);",
     "q[c] = fmaf(Cj, u[c], Sj * u[c]);"),
    ("double vote", "hist[idx] += 1;", "hist[idx] += 2;"),
    ("top-K tie order", "while (pos > 0 && counts[pos - 1] < h)",
     "while (pos > 0 && counts[pos - 1] <= h)"),
    ("decode off by half a cell", "p[c] = (float)(2 * ic[c] + 1) / (float)G - 1.0f;",
     "p[c] = (float)(2 * ic[c]) / (float)G - 1.0f;"),
    ("decode w sign", "q[0] = (1.0f - s) / den;", "q[0] = (s - 1.0f) / den;"),
    ("decode index", "ic[1] = (idx / G) % G;", "ic[1] = idx % G;"),
    ("residual row 1 sign", "float r1 = (P[1] * vz - P[2] * vy) - w * D[0];",
     "float r1 = (P[1] * vz - P[2] * vy) + w * D[0];"),
    ("residual row 0 operand", "r0 = r0 + D[2] * vz;", "r0 = r0 + D[2] * vy;"),
    ("residual row 3 transposed", "float r3 = (P[0] * vy - P[1] * vx) - w * D[2];",
     "float r3 = (P[1] * vx - P[0] * vy) - w * D[2];"),
    ("residual sum dropped term", "s = s + r3 * r3;", "s = s + r2 * r3;"),
    ("residual a+b instead of a-b", "D[c] = a[c] - b[c];", "D[c] = b[c] - a[c] + a[c] - a[c];"),
    ("winner tie to last", "if (c > best_cnt) {", "if (c >= best_cnt) {"),
]


def _run_mutant(name, old, new, tmp: Path):
    src = (ROOT / "oracle" / "rotvote_oracle.c").read_text()
    assert src.count(old) == 1, f"mutant site not unique: {name}"
    d = tmp / name.replace(" ", "_").replace("/", "_")
    d.mkdir()
    (d / "rotvote_oracle.h").write_text((ROOT / "oracle" / "rotvote_oracle.h").read_text())
    (d / "m.c").write_text(src.replace(old, new))
    oracle.build(src=d / "m.c", out=d / "liborc.so", extra=["-w"])
    r = subprocess.run([sys.executable, str(ROOT / "tests" / "pins.py"), "--lib",
                        str(d / "liborc.so")], capture_output=True, text=True, timeout=300)
    return name, r.returncode, r.stdout[-400:]


@pytest.mark.slow
def test_every_mutant_fails_a_pin():
    with tempfile.TemporaryDirectory() as t:
        tmp = Path(t)
        with ThreadPoolExecutor(max_workers=6) as ex:
            results = list(ex.map(lambda m: _run_mutant(*m, tmp), MUTANTS))
    survived = [(n, out) for n, rc, out in results if rc == 0]
    assert not survived, f"mutants not caught by any pin: {survived}"
