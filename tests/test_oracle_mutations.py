"""Mutation probe of the oracle's pins (CPU only).  Each mistake below is
planted in a copy of oracle.cpp, built into a library of its own and loaded
by the pin tests in a separate process (DV_ORACLE_LIB); at least one pin
must fail (or the mutant must crash under them).  The product path is not involved: this checks that the pins
would notice a plausible error in the oracle itself."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_CPP = os.path.join(ROOT, "oracle", "oracle.cpp")
PINS = ["tests/test_oracle_label.py", "tests/test_oracle_centroids.py", "tests/test_oracle_owner.py",
        "tests/test_oracle_edges.py", "tests/test_oracle_diff.py", "tests/test_oracle_events.py",
        "tests/test_oracle_geometry.py", "tests/test_oracle_weighted.py"]

# (name, text in oracle.cpp, planted replacement)
MUTATIONS = [
    ("rotated frame index", "pb = f[(2 * r + 7) & 7];", "pb = f[(2 * r + 6) & 7];"),
    ("first-neighbour rule without its diagonal check",
     "if (t != MAXLINK && pa != pb && t != ck)", "if (t != MAXLINK && t != ck)"),
    ("wrong inner-frame point", "const int INNER[4][2] = {{128, 128}, {-128, 128},",
     "const int INNER[4][2] = {{128, 128}, {128, 128},"),
    ("centre rounded down instead of half up",
     "qx[l] = (int32_t)pos_mod(256 * rx + floor_div(512 * sx[l] + n[l], 2 * n[l]), 256LL * lx);",
     "qx[l] = (int32_t)pos_mod(256 * rx + floor_div(512 * sx[l], 2 * n[l]), 256LL * lx);"),
    ("minimum image with the wrong half-width", "const int64_t h = L / 2;", "const int64_t h = (L + 1) / 2;"),
    ("ties to the highest label", "if (d < bd) { bd = d; best = i; }", "if (d <= bd) { bd = d; best = i; }"),
    ("now points with several preimages kept", "keepN[n] = cnt[n] == 1 ? 1 : 0;", "keepN[n] = cnt[n] >= 1 ? 1 : 0;"),
    ("vertex at two gaps", "if (gaps < 3) return;", "if (gaps < 2) return;"),
    ("MAXLINK frame points counted as gaps",
     "if (a != b && a != MAXLINK && b != MAXLINK) ++gaps;", "if (a != b) ++gaps;"),
    ("preimages not counted", "cnt[m] += 1;", "cnt[m] = 1;"),
    ("weighted: x sum without weights", "sx[l] += w * axis_off(x - rx, lx, ox);",
     "sx[l] += axis_off(x - rx, lx, ox);"),
    ("weighted: rounded down", "const __int128 num = (__int128)512 * S + W, den = (__int128)2 * W;",
     "const __int128 num = (__int128)512 * S, den = (__int128)2 * W;"),
    ("weighted: no clamp at one unit", "if (!(v >= 1.0)) return 1;", "if (!(v >= 0.0)) return 0;"),
    ("weighted: weight scale 1/128", "const double v = std::floor(256.0 * (double)rho + 0.5);",
     "const double v = std::floor(128.0 * (double)rho + 0.5);"),
    ("weighted: y offsets from the root's x", "sy[l] += w * axis_off(y - ry, ly, oy);",
     "sy[l] += w * axis_off(y - rx, ly, oy);"),
    ("weighted: truncating division", "if ((num % den) != 0 && num < 0) q -= 1;", ""),
]


@pytest.mark.parametrize("name,a,b", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_a_planted_mistake(name, a, b, tmp_path):
    src = open(ORACLE_CPP).read()
    assert src.count(a) == 1, f"mutation point of '{name}' not found once in oracle.cpp"
    mut = tmp_path / "oracle_mut.cpp"
    mut.write_text(src.replace(a, b))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-shared", "-fPIC", str(mut), "-o", str(lib)],
                   check=True, capture_output=True)
    env = dict(os.environ, DV_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *PINS], cwd=ROOT, env=env, capture_output=True, text=True)
    # a failed pin (1) or a crash of the mutant under the pins (negative: a
    # signal) both count; 0 is a survivor, 4 / 5 a broken run
    assert r.returncode not in (0, 4, 5), f"'{name}' survived the pins (rc {r.returncode}):\n{r.stdout[-2000:]}"
