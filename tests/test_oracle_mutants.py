"""Planted mistakes: every pin-suite run against a deliberately broken build of
the oracle must fail.

Each mutant is one plausible slip (a dropped term, a wrong sign, an index or
operand swapped, a strict test made loose) applied to a copy of
``oracle/seeds_oracle.c`` and compiled on the CPU into a temporary library.
The pin suite (tests/test_oracle_pins.py) then runs in a child process with
SEEDS_ORACLE_LIB naming that library and has to report a failure.
"""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))

# (name, text in the oracle source, replacement, which occurrence)
MUTANTS = [
    ("bin-divisor", "(c * B) / 256", "(c * B) / 255", 0),
    ("bin-channel-order", "(r * B + g) * B + b", "(b * B + g) * B + r", 0),
    ("grid-gy-floor", "(2 * (int64_t)K + gx) / (2 * (int64_t)gx)", "(int64_t)K / gx", 0),
    ("grid-label-transposed", "sy * gx + sx", "sx * gy + sy", 0),
    ("descend-index", "ux / 2]", "(ux + 1) / 2 < old_uw ? (ux + 1) / 2 : ux / 2]", 0),
    ("connect-any-edge", "return got == need;", "return got >= 1;", 0),
    ("candidates-no-west", "static const int dx[4] = {0, 1, 0, -1}, dy[4] = {-1, 0, 1, 0};",
     "static const int dx[4] = {0, 1, 0, 0}, dy[4] = {-1, 0, 1, 0};", 0),
    ("colour-gain-drop-one", "- (st->hist[(int64_t)k * st->nbins + j] - 1)",
     "- st->hist[(int64_t)k * st->nbins + j]", 0),
    ("boundary-gain-drop-one", "patch_count(st, ix, iy, n) + 1", "patch_count(st, ix, iy, n)", 0),
    ("boundary-gain-sign", "return plus - minus;", "return minus - plus;", 0),
    ("pixel-tie-larger-label", "g > best) { best = g; bn = cand[c]; }",
     "g >= best) { best = g; bn = cand[c]; }", 0),
    ("pixel-accept-loose", "d->accepted = best > 0;", "d->accepted = best >= 0;", 0),
    ("exact-gain-drop-term", "(hn[j] - hk[j] + hl[j])", "(hn[j] - hk[j])", 0),
    ("exact-accept-loose", "d->accepted = best > 0;", "d->accepted = best >= 0;", 1),
    ("intersect-max", "S += a < b ? a : b;", "S += a > b ? a : b;", 0),
    ("intersect-block-not-removed", "hkl[j] = hk[j] - hl[j];", "hkl[j] = hk[j];", 0),
    ("intersect-size-not-reduced", "int64_t Akl = st->size[k] - m;", "int64_t Akl = st->size[k];", 0),
    ("class-rows-cols-swapped", "for (int uy = cls / 3; uy < st->uh; uy += 3)",
     "for (int uy = cls % 3; uy < st->uh; uy += 3)", 0),
    ("apply-size-not-moved", "st->size[n] += 1;", "st->size[n] += 0;", 0),
    ("drop-rule-wrong-side", "is_source[dec[i].n]", "is_source[dec[i].k]", 0),
    ("energy-G-not-squared", "gs += (int64_t)cnts[i] * cnts[i];", "gs += (int64_t)cnts[i];", 0),
    ("sequential-column-order",
     "for (int uy = 0; uy < st->uh; ++uy)\n                for (int ux = 0; ux < st->uw; ++ux) {",
     "for (int ux = 0; ux < st->uw; ++ux)\n                for (int uy = 0; uy < st->uh; ++uy) {", 0),
    ("sequential-skips-half-the-moves", "if (d.accepted) apply_move(st, ux, uy, d.k, d.n);",
     "if (d.accepted && ((ux + uy) & 1)) apply_move(st, ux, uy, d.k, d.n);", 0),
]


def _mutate(src: str, old: str, new: str, occ: int) -> str:
    pos = -1
    for _ in range(occ + 1):
        pos = src.find(old, pos + 1)
        assert pos >= 0, f"mutation site not found: {old!r} #{occ}"
    return src[:pos] + new + src[pos + len(old):]


@pytest.mark.parametrize("name,old,new,occ", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new, occ, tmp_path):
    with open(oracle.SRC) as f:
        src = f.read()
    mutated = _mutate(src, old, new, occ)
    assert mutated != src
    c = tmp_path / "mutant.c"
    so = tmp_path / "libmutant.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-o", str(so), str(c)],
                   check=True)
    env = dict(os.environ, SEEDS_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-p", "no:xdist", "--timeout", "120",
                        os.path.join(HERE, "test_oracle_pins.py")],
                       env=env, capture_output=True, text=True, timeout=900, cwd=HERE)
    assert r.returncode != 0, f"mutant {name} survived the pin suite:\n{r.stdout[-2000:]}"
