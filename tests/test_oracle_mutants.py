"""The oracle's pins catch plausible mistakes: each case plants one mistake
(a dropped term, a wrong sign, constant or ratio) in a copy of the oracle's
source, builds it, and runs the pins that must then fail, in a child
process that loads the copy.  CPU only; the planted mistakes live in
temporary copies, never in the oracle itself."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "igks_oracle.c")

# name: (text in the oracle, its replacement, the pins that catch it: run
# together, they must fail)
MUTANTS = {
    "sutherland exponent 1": (
        "pow(th, 1.5)", "pow(th, 1.0)",
        ["tests/test_oracle_pins.py::test_sutherland_viscosity"]),
    "sutherland constant at 273.15 K": (
        "110.4 / 288.15", "110.4 / 273.15",
        ["tests/test_oracle_pins.py::test_sutherland_viscosity"]),
    "limiter without its minimum side": (
        "if (nmin < wc) { double r = (wmin - wc) / (nmin - wc); if (r < phi) phi = r; }", "",
        ["tests/test_oracle_pins.py::test_limiter_factor_by_hand"]),
    "limiter ratio inverted": (
        "if (nmax > wc) { double r = (wmax - wc) / (nmax - wc);",
        "if (nmax > wc) { double r = (nmax - wc) / (wmax - wc + 1e-300);",
        ["tests/test_oracle_pins.py::test_limiter_factor_by_hand"]),
    "Cp without the free-stream pressure": (
        "cp[w] = ((fx * nx + fy * ny) / S - c->p_inf) / q;", "cp[w] = ((fx * nx + fy * ny) / S) / q;",
        ["tests/test_oracle_pins.py::test_wall_loads_of_a_closed_box_at_rest"]),
    "Cp with the normal reversed": (
        "cp[w] = ((fx * nx + fy * ny) / S - c->p_inf) / q;", "cp[w] = ((-fx * nx - fy * ny) / S - c->p_inf) / q;",
        ["tests/test_oracle_pins.py::test_wall_loads_of_a_closed_box_at_rest"]),
    "lift with the sine sign flipped": (
        "*cl = (-Fx * sa + Fy * ca) / q;", "*cl = (Fx * sa + Fy * ca) / q;",
        ["tests/test_oracle_pins.py::test_wall_loads_rotate_with_mesh_and_stream"]),
    "lift of the opposite sign": (
        "*cl = (-Fx * sa + Fy * ca) / q;", "*cl = (Fx * sa - Fy * ca) / q;",
        ["tests/test_oracle_pins.py::test_wall_loads_of_a_floor_at_rest"]),
    "drag with the sine sign flipped": (
        "*cd = (Fx * ca + Fy * sa) / q;", "*cd = (Fx * ca - Fy * sa) / q;",
        ["tests/test_oracle_pins.py::test_wall_loads_of_a_floor_at_rest"]),
    "skin friction against the flow": (
        "if (tx * ca + ty * sa < 0) { tx = -tx; ty = -ty; }", "",
        ["tests/test_oracle_pins.py::test_plate_drag_is_its_skin_friction"]),
    "SA diagonal without its source part": (
        "+ ds + c->area[i] * so[3];", "+ ds;",
        ["tests/test_oracle_pins.py::test_sa_diagonal_assembly"]),
    "SA diagonal without its face part": (
        "+ ds + c->area[i] * so[3];", "+ c->area[i] * so[3];",
        ["tests/test_oracle_pins.py::test_sa_diagonal_assembly",
         "tests/test_oracle_solver.py::test_sa_lusgs_solves_factored_system"]),
    "SA wall increment not negated": (
        "dWg[3] = dWi[3]; dWg[4] = -dWi[4];\n    } else {", "dWg[3] = dWi[3]; dWg[4] = dWi[4];\n    } else {",
        ["tests/test_oracle_solver.py::test_sa_lusgs_solves_factored_system"]),
    "sweep blocks ignored in the forward sweep": (
        "const int cross = c->sblk && c->sblk[j] != c->sblk[i];",
        "const int cross = 0;",
        ["tests/test_oracle_solver.py::test_lusgs_solves_factored_system"]),
    "second block pass without the cross-block terms": (
        "lusgs_pass(c, c->dW1);", "lusgs_pass(c, NULL);",
        ["tests/test_oracle_solver.py::test_lusgs_solves_factored_system"]),
    "second block pass takes its own cross-block increments": (
        "const double *dj = cross ? &dWx[5 * j] : &dW[5 * j];", "const double *dj = &dW[5 * j];",
        ["tests/test_oracle_solver.py::test_lusgs_solves_factored_system"]),
    "sweep blocks ignored in the backward sweep": (
        "if (j <= i) continue;\n                if (c->sblk && c->sblk[j] != c->sblk[i]) continue;",
        "if (j <= i) continue;",
        ["tests/test_oracle_solver.py::test_lusgs_solves_factored_system"]),
    "SA lower neighbour subtracted": (
        "&W[5 * j], nx, ny, S, face_rn(c, f), &dg, &of);\n                acc[4] += of * dj[4];",
        "&W[5 * j], nx, ny, S, face_rn(c, f), &dg, &of);\n                acc[4] -= of * dj[4];",
        ["tests/test_oracle_solver.py::test_sa_lusgs_solves_factored_system"]),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_its_pins(name, tmp_path):
    old, new, pins = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"the text to mutate must occur once: {old!r}"
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                    "-o", str(lib), str(mutant), "-lm"], check=True)
    env = dict(os.environ, OIGKS_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, f"{name}: {pins} did not fail\n{r.stdout[-2000:]}"
