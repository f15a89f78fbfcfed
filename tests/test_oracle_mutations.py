"""The oracle pins are sharp: plausible mistakes planted in copies of the
oracle (on the CPU, never on the GPU) must each fail at least one pin.

Every mutant is a one-line change of the kind a reader might make when
writing the method from the paper: a weight sign in the radical plane
(Sec. 4.2, Eq. 2), a dropped factor, a transposed operand in the vertex
solve, a box face on the wrong side, a wrong tetrahedron centroid weight, a
clockwise facet, a premature stop of the candidate walk, a squared radius,
a fan without its reference point, the wrong winner among coincident sites;
for the dual tetrahedra read off the cells, box vertices kept, every cell
listing the tetrahedron, the vertices of the wrong cell; and for the
robustness margin that decides which cells the bit-exact gate covers, a
constant margin, box faces left out, the vertex error scale left out, and the
weight shift of the empty-cell certificate with the wrong sign.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "weight_sign": ("h.b = 0.5 * (d2 + (site_w(in, i) - site_w(in, j)));",
                    "h.b = 0.5 * (d2 + (site_w(in, j) - site_w(in, i)));"),
    "drop_half": ("h.b = 0.5 * (d2 + (site_w(in, i) - site_w(in, j)));",
                  "h.b = (d2 + (site_w(in, i) - site_w(in, j)));"),
    "cramer_swap": ("y[k] = (A.b * bc[k] + B.b * ca[k] + C.b * ab[k]) / det;",
                    "y[k] = (A.b * bc[k] + B.b * ab[k] + C.b * ca[k]) / det;"),
    "box_sign": ("lo.b = p[ax] - box[ax];", "lo.b = box[ax] - p[ax];"),
    "centroid_weight": ("mom[r] += det * (a0[r] + a1[r] + a2[r]) / 4.0;",
                        "mom[r] += det * (a0[r] + a1[r] + a2[r]) / 3.0;"),
    "clockwise_facets": ("std::sort(ang.begin(), ang.end());", "std::sort(ang.rbegin(), ang.rend());"),
    "early_stop": ("if (c.d > R) break;", "if (c.d > 0.7 * R) break;"),
    "coincident_tie": ("if (wt > ww || (wt == ww && ord[t] < ord[win])) win = t;",
                       "if (wt > ww || (wt == ww && ord[t] > ord[win])) win = t;"),
    "squared_radius": ("return std::sqrt(r2);\n}", "return r2;\n}"),
    "fan_without_reference": ("a0[r] = f0[r] - ref[r];", "a0[r] = f0[r];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "vd_oracle.cpp")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, "mutation site moved"
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("__init__.py", "brute.py"):
        shutil.copy(os.path.join(ROOT, "oracle", f), pkg / f)
    (pkg / "vd_oracle.cpp").write_text(src.replace(old, new))
    subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o",
                    str(pkg / "liboracle.so"), str(pkg / "vd_oracle.cpp")], check=True)
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(1, %r); import pytest; "
            "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', '--import-mode=append', %r]))"
            % (str(tmp_path), ROOT, os.path.join(ROOT, "tests", "test_oracle_pins.py")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=str(tmp_path),
                       timeout=600)
    assert r.returncode == 1, "mutant %s survived the pins:\n%s" % (name, r.stdout[-2000:])


# Mistakes in the analytic gradient oracle (the transport of the volume and
# moment integrals, the vertex solve, the chain to sites and weights).
GRAD_MUTANTS = {
    "moment_sign": ("dA[c] += -(alpha * AY + S @ gamma) / D", "dA[c] += -(alpha * AY - S @ gamma) / D"),
    "weight_half_sign": ("add(c, gp, -0.5 * dB[c])", "add(c, gp, 0.5 * dB[c])"),
    "vertex_normal_term": ("dA[c] += -g[k] * y[v]", "dA[c] += g[k] * y[v]"),
    "centroid_quotient": ("alpha = g_vol - gc @ m / (V * V)", "alpha = g_vol"),
    "box_face_sign": ("add(i, -dB[c] * a, 0.0)", "add(i, dB[c] * a, 0.0)"),
    "transposed_solve": ("g = np.linalg.solve(M.T, gv[v])", "g = np.linalg.solve(M, gv[v])"),
    "pyramid_moment": ("integ[c][1] / (4.0 * np.linalg.norm", "integ[c][1] / (3.0 * np.linalg.norm"),
    "moving_box_face_sign": ("gp[j, ax] += box_db[c] if side else -box_db[c]", "gp[j, ax] += box_db[c]"),
}


@pytest.mark.parametrize("name", sorted(GRAD_MUTANTS))
def test_planted_gradient_mistake_is_caught(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "grad.py")).read()
    old, new = GRAD_MUTANTS[name]
    assert src.count(old) == 1, "mutation site moved"
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("__init__.py", "brute.py", "vd_oracle.cpp"):
        shutil.copy(os.path.join(ROOT, "oracle", f), pkg / f)
    (pkg / "grad.py").write_text(src.replace(old, new))
    subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o",
                    str(pkg / "liboracle.so"), str(pkg / "vd_oracle.cpp")], check=True)
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(1, %r); import pytest; "
            "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', '--import-mode=append', %r]))"
            % (str(tmp_path), ROOT, os.path.join(ROOT, "tests", "test_oracle_grad.py")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=str(tmp_path),
                       timeout=600)
    assert r.returncode == 1, "mutant %s survived the pins:\n%s" % (name, r.stdout[-2000:])


# Mistakes in reading the dual tetrahedra off the cells.
DUAL_MUTANTS = {
    "box_vertices_kept": ("            if c[0] > i:\n", "            if c[2] > i:\n"),
    "listed_by_every_cell": ("            if c[0] > i:\n", "            if c[0] >= 0:\n"),
    "neighbouring_cell": ('codes = res["vert_code"][res["vert_off"][t]:res["vert_off"][t + 1]]',
                          'codes = res["vert_code"][res["vert_off"][t]:res["vert_off"][min(t + 2, len(res["ids"]))]]'),
}


@pytest.mark.parametrize("name", sorted(DUAL_MUTANTS))
def test_planted_dual_mistake_is_caught(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "__init__.py")).read()
    old, new = DUAL_MUTANTS[name]
    assert src.count(old) == 1, "mutation site moved"
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("brute.py", "grad.py", "vd_oracle.cpp"):
        shutil.copy(os.path.join(ROOT, "oracle", f), pkg / f)
    (pkg / "__init__.py").write_text(src.replace(old, new))
    subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o",
                    str(pkg / "liboracle.so"), str(pkg / "vd_oracle.cpp")], check=True)
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(1, %r); import pytest; "
            "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', '--import-mode=append', %r]))"
            % (str(tmp_path), ROOT, os.path.join(ROOT, "tests", "test_oracle_dual.py")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=str(tmp_path),
                       timeout=600)
    assert r.returncode == 1, "mutant %s survived the pins:\n%s" % (name, r.stdout[-2000:])


# Mistakes in the robustness margin (which cells the bit-exact gate covers)
# and in the certificate of empty power cells.
MARGIN_MUTANTS = {
    "constant_margin": ("return std::max(margin, 0.0);", "return tau_m;"),
    "margin_without_box_faces": ("for (const Plane& h : boxp.pl) visit(h);", ""),
    "margin_without_vertex_error": ("double sigma = ev[k] + norm3(v.y) + dk;", "double sigma = norm3(v.y) + dk;"),
    "empty_certificate_shift_sign": ("h.b += 0.5 * wshift;", "h.b -= 0.5 * wshift;"),
}


@pytest.mark.parametrize("name", sorted(MARGIN_MUTANTS))
def test_planted_margin_mistake_is_caught(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "vd_oracle.cpp")).read()
    old, new = MARGIN_MUTANTS[name]
    assert src.count(old) == 1, "mutation site moved"
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("__init__.py", "brute.py", "grad.py"):
        shutil.copy(os.path.join(ROOT, "oracle", f), pkg / f)
    (pkg / "vd_oracle.cpp").write_text(src.replace(old, new))
    subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o",
                    str(pkg / "liboracle.so"), str(pkg / "vd_oracle.cpp")], check=True)
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(1, %r); import pytest; "
            "sys.exit(pytest.main(['-q', '-p', 'no:cacheprovider', '--import-mode=append', %r]))"
            % (str(tmp_path), ROOT, os.path.join(ROOT, "tests", "test_oracle_margin.py")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=str(tmp_path),
                       timeout=600)
    assert r.returncode == 1, "mutant %s survived the margin pins:\n%s" % (name, r.stdout[-2000:])


# Mistakes in the k-d tree candidate mode (its node key must never exceed
# the plane distance of a site below the node).
KD_MUTANTS = {
    "node_key_ignores_weights": ("const double c = std::min(0.0, wi - nd.wmax) * (1.0 + tau);",
                                 "const double c = 0.0;"),
    "node_key_full_distance": ("else lb = 0.5 * dB * (1.0 - tau);", "else lb = dB * (1.0 - tau);"),
}


@pytest.mark.parametrize("name", sorted(KD_MUTANTS))
def test_planted_kdtree_mistake_is_caught(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "vd_oracle.cpp")).read()
    old, new = KD_MUTANTS[name]
    assert src.count(old) == 1, "mutation site moved"
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("__init__.py", "brute.py", "grad.py"):
        shutil.copy(os.path.join(ROOT, "oracle", f), pkg / f)
    (pkg / "vd_oracle.cpp").write_text(src.replace(old, new))
    subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o",
                    str(pkg / "liboracle.so"), str(pkg / "vd_oracle.cpp")], check=True)
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(1, %r); import pytest; "
            "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', '--import-mode=append', %r]))"
            % (str(tmp_path), ROOT, os.path.join(ROOT, "tests", "test_oracle_kdtree.py")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=str(tmp_path),
                       timeout=600)
    assert r.returncode == 1, "mutant %s survived the k-d tree tests:\n%s" % (name, r.stdout[-2000:])
