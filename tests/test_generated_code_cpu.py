"""The emitted HIP straight-line code, executed on the CPU, equals the exact
tables: the b-form (monomial coefficients from the gathered coefficients,
with factored pair sums) and the w-form (per-site weights) of every
sub-region, about the sub-region's origin, and the sub-region selection.
This pins the code generator's text, not only its data."""

import re
from fractions import Fraction

import numpy as np
import pytest

from paper_2102_08514_amd.gen.interp import orbit_of
from paper_2102_08514_amd.gen.tables import GENERATED, load

NAMES = ["bcc_linear", "cc_zp", "bcc_quartic", "fcc_6dir", "d4s_8dir", "d4_8dir", "cc_tp2", "cc_tp3", "cc_tp4",
         "cc_linear_rd", "bcc_quintic_rd", "bcc_voronoi1", "fcc_voronoi1", "cc_bcc_voronoi1", "cc_fcc_voronoi1",
         "fcc_voronoi2", "cc_fcc_voronoi2"]


def _functions(text):
    """{name: body lines} for the b_k / w_k / origin device functions."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"static (?:void|AT|int) (b_\d+|w_\d+|origin|orbit)\(", line)
        if m:
            cur = m.group(1)
            out[cur] = []
            continue
        if cur is not None:
            if line.startswith("  }"):
                cur = None
            else:
                out[cur].append(line.strip())
    return out


def _lit(s):
    return float(s)


def run_b(lines, c):
    env = {f"x{r}": v for r, v in enumerate(c)}
    b = {}
    for ln in lines:
        if ln.startswith("const AT x") and "g.template" in ln:
            continue
        m = re.match(r"const AT (x\d+) = fma\((x\d+), AT\(([^)]+)\), (x\d+)\);", ln)
        if m:
            env[m.group(1)] = env[m.group(2)] * _lit(m.group(3)) + env[m.group(4)]
            continue
        m = re.match(r"b\[(\d+)\] = (x\d+) \* AT\(([^)]+)\);", ln)
        if m:
            b[int(m.group(1))] = env[m.group(2)] * _lit(m.group(3))
            continue
        m = re.match(r"b\[(\d+)\] = fma\((x\d+), AT\(([^)]+)\), b\[\d+\]\);", ln)
        if m:
            b[int(m.group(1))] += env[m.group(2)] * _lit(m.group(3))
            continue
        m = re.match(r"b\[(\d+)\] = AT\(0\);", ln)
        if m:
            b[int(m.group(1))] = 0.0
            continue
        raise AssertionError(f"unparsed line: {ln}")
    return b


def run_w(lines, mono):
    env = {}
    sym = lambda s: mono[int(s[5:-1])] if s.startswith("mono[") else env[s]  # noqa: E731
    w, cur = [], None
    for ln in lines:
        m = re.match(r"const AT (y\d+) = fma\((\S+), AT\(([^)]+)\), (\S+)\);", ln)
        if m:
            env[m.group(1)] = sym(m.group(2)) * _lit(m.group(3)) + sym(m.group(4))
            continue
        m = re.match(r"\{ AT wv = (\S+) \* AT\(([^)]+)\);", ln)
        if m:
            cur = sym(m.group(1)) * _lit(m.group(2))
            continue
        m = re.match(r"wv = fma\((\S+), AT\(([^)]+)\), wv\);", ln)
        if m:
            cur += sym(m.group(1)) * _lit(m.group(2))
            continue
        m = re.match(r"g\.template put<([-\d, ]+)>\(wv\); \}", ln)
        if m:
            w.append((tuple(int(v) for v in m.group(1).split(",")), cur))
            continue
        raise AssertionError(f"unparsed line: {ln}")
    return w


@pytest.mark.parametrize("name", NAMES)
def test_emitted_code_matches_tables(name):
    t = load(name)
    text = open(f"{GENERATED}/{name}.inc").read()
    fn = _functions(text)
    mons = t.monomials()
    rng = np.random.default_rng(5)
    # origins per sub-region, from the emitted origin() selector
    orig_lines = fn["origin"]
    for k, orb in enumerate(t.orbits):
        origin = []
        for d in range(t.s):
            line = next(ln for ln in orig_lines if ln.startswith(f"if (d == {d})"))
            vals = [float(v) for v in re.findall(r"AT\(([-0-9.e]+)\)", line)]
            # nested selector: value for ob == k is the k-th literal (last one is the default)
            origin.append(vals[k] if k < len(vals) else vals[-1])
        stencil = orb["stencil"]
        # random gathered values and a random point: psi two ways
        c = rng.uniform(-1, 1, len(stencil))
        u = rng.uniform(0, t.D / 2, t.s)
        z = u - np.array(origin)
        b = run_b(fn[f"b_{k}"], c)
        psi_code = sum(b.get(m, 0.0) * np.prod(z ** np.array(e)) for m, e in enumerate(mons))
        psi_tab = sum(ci * float(P(tuple(Fraction(float(v)) for v in u))) for ci, P in zip(c, orb["polys"]))
        assert abs(psi_code - psi_tab) < 1e-12, (k, psi_code, psi_tab)
        mono = [float(np.prod(z ** np.array(e))) for e in mons]
        w = run_w(fn[f"w_{k}"], mono)
        assert [j for j, _ in w] == [tuple(j) for j in stencil]
        for (j, wv), P in zip(w, orb["polys"]):
            assert abs(wv - float(P(tuple(Fraction(float(v)) for v in u)))) < 1e-12


def _selector(body):
    """The emitted orbit() body as a Python function of the folded point."""
    src = ["def orbit(up):"]
    for ln in body:
        m = re.match(r"int code = 0;", ln)
        if m:
            src.append("    code = 0")
            continue
        m = re.match(r"code \|= \(\((.*)\) - AT\(([-0-9.e]+)\) (>=|>) AT\(0\)\) \? (\d+) : 0;", ln)
        if m:
            terms = re.sub(r"AT\((-?\d+)\)", r"(\1)", m.group(1))
            src.append(f"    code |= {m.group(4)} if (({terms}) - Fraction({m.group(2)!r}) {m.group(3)} 0) else 0")
            continue
        m = re.match(r"const unsigned idx = static_cast<unsigned>\(code\) % (\d+)u;", ln)
        if m:
            src.append(f"    idx = code % {m.group(1)}")
            continue
        m = re.match(r"const unsigned long long word = (.*);", ln)
        if m:
            # a right-nested chain (idx < T1u ? W1ull : (idx < T2u ? W2ull : ... Wnull))
            e = m.group(1)
            thr = [int(v) for v in re.findall(r"idx < (\d+)u", e)]
            words = [int(v) for v in re.findall(r"(\d+)ull", e)]
            assert len(words) == len(thr) + 1
            src.append(f"    word = next((w for t, w in zip({thr}, {words[:-1]}) if idx < t), {words[-1]})")
            continue
        m = re.match(r"return static_cast<int>\(\(word >> \((\d+) \* \(idx % (\d+)u\)\)\) & (\d+)ull\);", ln)
        if m:
            src.append(f"    return (word >> ({m.group(1)} * (idx % {m.group(2)}))) & {m.group(3)}")
            continue
        m = re.match(r"return static_cast<int>\(\((\d+)ull >> \(4 \* code\)\) & 15ull\);", ln)
        if m:
            src.append(f"    return ({m.group(1)} >> (4 * code)) & 15")
            continue
        raise AssertionError(f"unparsed line: {ln}")
    env = {"Fraction": Fraction}
    exec("\n".join(src), env)
    return env["orbit"]


@pytest.mark.parametrize("name", ["fcc_6dir", "d4s_8dir", "d4_8dir", "bcc_voronoi1", "fcc_voronoi1",
                                  "cc_bcc_voronoi1", "fcc_voronoi2"])
def test_emitted_subregion_selector(name):
    """The emitted selector (plane bits with their tie sides, then the packed
    table or sigma(q mod r) of Sec. 4.2) gives the sub-region of the exact
    tables, also for points exactly on splitting planes (dyadic grid points),
    where it must name a sub-region whose closure holds the point."""
    from paper_2102_08514_amd.gen.analysis import chamber_constraints, chamber_vertices
    from paper_2102_08514_amd.gen.select import tie_point
    t = load(name)
    text = open(f"{GENERATED}/{name}.inc").read()
    orbit = _selector(_functions(text)["orbit"])
    rng = np.random.default_rng(6)
    h = Fraction(t.D, 2)
    F = chamber_constraints(t.s, t.fold, h)
    g = tie_point(t.planes, F, chamber_vertices(t.s, t.fold, h))
    on_plane = 0
    for trial in range(1500):
        if trial % 2:
            u = sorted(rng.uniform(0, t.D / 2, t.s), reverse=True)
            up = [Fraction(v) for v in u]
        else:
            u = sorted((Fraction(int(v), 8) for v in rng.integers(0, 4 * t.D + 1, t.s)), reverse=True)
            up = list(u)
        if t.fold == "D" and rng.random() < 0.5:
            up[-1] = -up[-1]
        if not all(sum(Fraction(a) * x for a, x in zip(row, up)) + c >= 0 for row, c in F):
            continue
        got = orbit(up)
        assert got == orbit_of(t, up)
        vals = [sum(a * b for a, b in zip(nu, up)) - off for nu, off in t.planes]
        if any(v == 0 for v in vals):
            on_plane += 1
            # the named sub-region's closure holds the point: just off the
            # point, toward the tie point, the plain selection agrees
            q = [a + Fraction(1, 10 ** 9) * (b - a) for a, b in zip(up, g)]
            assert all(sum(a * b for a, b in zip(nu, q)) != off for nu, off in t.planes)
            assert orbit_of(t, q) == got
    if t.planes:
        assert on_plane > 20

