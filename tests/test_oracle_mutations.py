"""The pins catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of oracle/lk_oracle.c (a dropped
term, a wrong sign, index or weight, a transposed operand, a changed
border, threshold or rounding rule), builds it, and runs the oracle pins
against it in a subprocess: the pins must fail for every mutant.  Runs on
the CPU only; the planted copies never leave a temporary directory.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lk_oracle.c")

MUTANTS = [
    ("Scharr x sign", "gx[(size_t)y * w + x] = (3.0 * (P(ym, xp) - P(ym, xm))",
     "gx[(size_t)y * w + x] = (3.0 * (P(ym, xm) - P(ym, xp))"),
    ("Scharr centre weight", "+ 10.0 * (P(y, xp) - P(y, xm))", "+ 9.0 * (P(y, xp) - P(y, xm))"),
    ("Scharr y uses x offsets", "gy[(size_t)y * w + x] = (3.0 * (P(yp, xm) - P(ym, xm))",
     "gy[(size_t)y * w + x] = (3.0 * (P(yp, xp) - P(ym, xm))"),
    ("binomial weights", "{1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16}",
     "{1.0 / 16, 5.0 / 16, 4.0 / 16, 5.0 / 16, 1.0 / 16}"),
    ("decimation phase", "int sy = reflect101(2 * y + j - 2, sh);", "int sy = reflect101(2 * y + j - 1, sh);"),
    ("reflect-101 replaced by symmetric", "if (i < 0) i = -i;", "if (i < 0) i = -i - 1;"),
    ("level size floor", "ws[l] = (ws[l - 1] + 1) / 2;", "ws[l] = ws[l - 1] / 2;"),
    ("bilinear x/y weights swapped",
     "return (1.0 - a) * (1.0 - b) * img[(size_t)ya * w + xa] + a * (1.0 - b) * img[(size_t)ya * w + xb]",
     "return (1.0 - a) * (1.0 - b) * img[(size_t)ya * w + xa] + b * (1.0 - a) * img[(size_t)ya * w + xb]"),
    ("bilinear tap not clamped low", "int xa = clampi(x0, 0, w - 1)", "int xa = clampi(x0, 1, w - 1)"),
    ("normal matrix cross term dropped", "Gxx += ax * ax; Gxy += ax * ay; Gyy += ay * ay;",
     "Gxx += ax * ax; Gxy += 0.0; Gyy += ay * ay;"),
    ("2x2 solve transposed", "double ex = (Gyy * bx - Gxy * by) / det;", "double ex = (Gxx * bx - Gxy * by) / det;"),
    ("mismatch sign", "bx += e * s->Gx[i * win + j];", "bx -= e * s->Gx[i * win + j];"),
    ("update sign", "dx += ex; dy += ey;", "dx -= ex; dy -= ey;"),
    ("level propagation without doubling", "gx = 2.0 * (gx + dx); gy = 2.0 * (gy + dy);",
     "gx = (gx + dx); gy = (gy + dy);"),
    ("template at the wrong scale", "const double cx = px * sc, cy = py * sc;",
     "const double cx = px * sc * 0.999, cy = py * sc;"),
    ("eigenvalue normalisation", "double meig = lam / ((double)nw * 255.0 * 255.0);",
     "double meig = lam / ((double)nw * 255.0);"),
    ("largest instead of smallest eigenvalue", "double lam = 0.5 * (Gxx + Gyy - sqrt(",
     "double lam = 0.5 * (Gxx + Gyy + sqrt("),
    ("residual without |.|", "acc += fabs(s->T[i * win + j]", "acc += (s->T[i * win + j]"),
    ("residual not averaged", "*res = acc / nw;", "*res = acc / win;"),
    ("convergence on the squared norm", "if (nrm < prm->eps) break;", "if (nrm * nrm < prm->eps) break;"),
    ("forward-backward threshold ignored", "if (fbd > prm->fb_thresh) st = LKO_LOST_FB;",
     "if (fbd > 1e9) st = LKO_LOST_FB;"),
    ("final in-image check dropped", "    if (!(bd >= 0.0)) return LKO_LOST_OOB;\n    return LKO_OK;",
     "    return LKO_OK;"),
    ("binary16 rounding truncates", "double r = nearbyint(x / q) * q;", "double r = trunc(x / q) * q;"),
    ("guess scaled to the wrong level", "double sc = ldexp(1.0, -(L - 1));", "double sc = ldexp(1.0, -L);"),
    # the decision margins (they decide which points the GPU parity rule treats as near a threshold)
    ("convergence margin from the last step only", "if (mc < m->conv) m->conv = mc;", "m->conv = mc;"),
    ("convergence margin in px instead of relative to eps", "double mc = fabs(nrm / prm->eps - 1.0);",
     "double mc = fabs(nrm - prm->eps);"),
    ("out-of-bounds margin of a level in level-0 px",
     "double bd = box_dist(qx, qy, -h, W - 1.0 + h, H - 1.0 + h);\n            if (fabs(bd) < m->oob) m->oob = fabs(bd);",
     "double bd = box_dist(qx, qy, -h, W - 1.0 + h, H - 1.0 + h);\n"
     "            if (fabs(bd) / sc < m->oob) m->oob = fabs(bd) / sc;"),
    ("out-of-bounds margin against the image box on every level",
     "double bd = box_dist(qx, qy, -h, W - 1.0 + h, H - 1.0 + h);\n            if (fabs(bd) < m->oob) m->oob = fabs(bd);",
     "double bd = box_dist(qx, qy, -h, W - 1.0 + h, H - 1.0 + h);\n"
     "            { double bi = box_dist(qx, qy, 0.0, W - 1.0, H - 1.0); if (fabs(bi) < m->oob) m->oob = fabs(bi); }"),
    ("out-of-bounds margin of the final check dropped",
     "double bd = box_dist(qx, qy, 0.0, J->w[0] - 1.0, J->h[0] - 1.0);\n    if (fabs(bd) < m->oob) m->oob = fabs(bd);",
     "double bd = box_dist(qx, qy, 0.0, J->w[0] - 1.0, J->h[0] - 1.0);"),
    ("forward-backward margin measured from q", "m.fb = fabs(fbd - prm->fb_thresh);",
     "m.fb = fabs(sqrt((bx - qx) * (bx - qx) + (by - qy) * (by - qy)) - prm->fb_thresh);"),
    ("forward-backward margin relative", "m.fb = fabs(fbd - prm->fb_thresh);", "m.fb = fabs(fbd / prm->fb_thresh - 1.0);"),
    ("eigenvalue margin absolute", "double me = fabs(meig / prm->min_eig - 1.0);", "double me = fabs(meig - prm->min_eig);"),
]

GFTT_MUTANTS = [
    ("gftt Scharr centre weight", "+ 10 * (Q(y, xp) - Q(y, xm))", "+ 9 * (Q(y, xp) - Q(y, xm))"),
    ("gftt Scharr y column", "10 * (Q(yp, x) - Q(ym, x))", "10 * (Q(yp, xm) - Q(ym, x))"),
    ("gftt tensor cross term dropped", "b += (long long)gx[o] * gy[o];", "b += 0;"),
    ("gftt largest eigenvalue", "resp[(size_t)y * w + x] = (tr - s) * 0.5;", "resp[(size_t)y * w + x] = (tr + s) * 0.5;"),
    ("gftt block one column short", "for (int i = -r; i <= r; ++i) {", "for (int i = -r; i < r; ++i) {"),
    ("gftt quality threshold ignored", "if (!(v > thr) || !(v > 0.0)) continue;", "if (!(v > 0.0)) continue;"),
    ("gftt no non-maximum suppression", "R[(size_t)yy * w + xx] > v) { peak = 0; break; }",
     "R[(size_t)yy * w + xx] > 1e300) { peak = 0; break; }"),
    ("gftt ascending rank", "if (a->r > b->r) return -1;\n    if (a->r < b->r) return 1;",
     "if (a->r < b->r) return -1;\n    if (a->r > b->r) return 1;"),
    ("gftt min distance not squared", "long long md2 = (long long)min_dist * min_dist;", "long long md2 = min_dist;"),
    ("gftt occupied points ignored", "if (dx * dx + dy * dy < (double)md2) ok = 0;", "if (dx * dx + dy * dy < 0.0) ok = 0;"),
    ("gftt border not applied", "for (int y = border; y < h - border; ++y)", "for (int y = 0; y < h; ++y)"),
]

PINS = ["tests/test_oracle_primitives.py", "tests/test_oracle_tracker.py", "tests/test_oracle_margins.py",
        "tests/test_oracle_cross.py", "tests/test_oracle_gftt.py"]

# planted in a copy of oracle/pool.py (the track-pool lifecycle)
POOL_SRC = os.path.join(ROOT, "oracle", "pool.py")
POOL_MUTANTS = [
    ("pool carry keeps the lost points", "keep = np.asarray(status) == OK", "keep = np.asarray(status) != OK"),
    ("pool top-up ignores the survivors' count", "room = max(int(target) - s, 0)", "room = max(int(target), 0)"),
    ("pool top-up ignores the survivors' positions", "occupied=surv_pts if s else None)", "occupied=None)"),
    ("pool identities for gated-out candidates", "        if not keep[i]:\n            continue\n", ""),
    ("pool identities restart at zero", "nid = int(next_id)", "nid = 0"),
    ("pool gate ignored", "keep = np.ones(n, bool) if gate_status is None else (np.asarray(gate_status) == OK)",
     "keep = np.ones(n, bool)"),
    ("pool stats carried/new swapped", "stats = (n0, len(si), len(ci) - len(si), len(ids))",
     "stats = (n0, len(ci) - len(si), len(si), len(ids))"),
]


@pytest.fixture(scope="module")
def workdir():
    with tempfile.TemporaryDirectory() as d:
        yield d


def test_unmutated_copy_passes(workdir):
    so = os.path.join(workdir, "ok.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", so, SRC, "-lm", "-lpthread"])
    env = dict(os.environ, LKO_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name,old,new", MUTANTS + GFTT_MUTANTS, ids=[m[0] for m in MUTANTS + GFTT_MUTANTS])
def test_pins_catch_mutant(workdir, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation site not found: " + name
    src = os.path.join(workdir, "mut.c")
    so = os.path.join(workdir, "mut_%d.so" % (abs(hash(name)) % 10 ** 8))
    open(src, "w").write(text.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-ffp-contract=off",
                           "-w", "-o", so, src, "-lm", "-lpthread"])
    env = dict(os.environ, LKO_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch: " + name

# planted in a copy of oracle/epipolar.py (the epipolar check)
EPI_SRC = os.path.join(ROOT, "oracle", "epipolar.py")
EPI_MUTANTS = [
    ("epipolar system rows transposed", "np.stack([np.kron(xq[i], xp[i])", "np.stack([np.kron(xp[i], xq[i])"),
    ("epipolar model left in normalized coordinates", "f = ki.T @ e @ ki", "f = e"),
    ("epipolar line normalised with its offset", "np.sqrt(l[:, 0] ** 2 + l[:, 1] ** 2)",
     "np.sqrt(l[:, 0] ** 2 + l[:, 1] ** 2 + l[:, 2] ** 2)"),
    ("epipolar error measured at p", "np.sum(hom(q) * l, axis=1)", "np.sum(hom(p) * l, axis=1)"),
    ("epipolar rank test dropped", "if len(sample) != 8 or sv[7] <= RANK_TOL * sv[0]:", "if len(sample) != 8:"),
    ("epipolar ties to the highest index", "key=lambda i: (counts[i], -i)", "key=lambda i: (counts[i], i)"),
]


def run_planted(src_path, env_name, test_file):
    env = dict(os.environ, **{env_name: src_path})
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", test_file],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


@pytest.mark.parametrize("name,old,new", EPI_MUTANTS, ids=[m[0] for m in EPI_MUTANTS])
def test_epipolar_pins_catch_mutant(workdir, name, old, new):
    text = open(EPI_SRC).read()
    assert text.count(old) == 1, "mutation site not found: " + name
    src = os.path.join(workdir, "epi_mut_%d.py" % (abs(hash(name)) % 10 ** 8))
    open(src, "w").write(text.replace(old, new))
    r = run_planted(src, "LKO_EPI_SRC", "tests/test_oracle_epipolar.py")
    assert r.returncode != 0, "pins did not catch: " + name


def test_unplanted_epipolar_copy_passes(workdir):
    src = os.path.join(workdir, "epi_copy.py")
    open(src, "w").write(open(EPI_SRC).read())
    r = run_planted(src, "LKO_EPI_SRC", "tests/test_oracle_epipolar.py")
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name,old,new", POOL_MUTANTS, ids=[m[0] for m in POOL_MUTANTS])
def test_pool_pins_catch_mutant(workdir, name, old, new):
    text = open(POOL_SRC).read()
    assert text.count(old) == 1, "mutation site not found: " + name
    src = os.path.join(workdir, "pool_mut_%d.py" % (abs(hash(name)) % 10 ** 8))
    open(src, "w").write(text.replace(old, new))
    env = dict(os.environ, LKO_POOL_SRC=src)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_pool.py"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch: " + name


def test_unplanted_pool_copy_passes(workdir):
    src = os.path.join(workdir, "pool_copy.py")
    open(src, "w").write(open(POOL_SRC).read())
    env = dict(os.environ, LKO_POOL_SRC=src)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_pool.py"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:]
