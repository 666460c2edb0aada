"""The renderer pins must catch plausible mistakes.  Each case below builds a
copy of the oracle with one deliberate error (a dropped cosine, a wrong area
factor, a wrong disc radius or height of the cosine-weighted bounce, an
inverted index ratio or a flipped sign in the refracted direction; in the
differentiable renderer of Eq. 9 a wrong sign of the hit point's motion, of an
edge's speed, a wrong edge length or speed), loads it in a child process and
checks that the pin aimed at that step fails there.  The
broken copies live in a temporary directory and are never used elsewhere."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    # next-event estimation of an area light
    "area_light_no_cos_l": ("float G = ((cx * cl) * area) / dist2;", "float G = (cx * area) / dist2;",
                            "tests/test_oracle_scatter.py::test_area_light_form_factor"),
    "area_light_no_area": ("float G = ((cx * cl) * area) / dist2;", "float G = (cx * cl) / dist2;",
                           "tests/test_oracle_scatter.py::test_area_light_form_factor"),
    # cosine-weighted bounce
    "bounce_disc_radius": ("float r = sqrtf(u1);", "float r = u1;",
                           "tests/test_oracle_scatter.py::test_cosine_bounce_form_factor"),
    "bounce_height": ("lz = sqrtf(1.0f - u1);", "lz = 1.0f - u1;",
                      "tests/test_oracle_scatter.py::test_cosine_bounce_distribution"),
    # refraction
    "refract_inverted_eta": ("float rel = ei / et;", "float rel = et / ei;",
                             "tests/test_oracle_scatter.py::test_refraction_obeys_snell"),
    "refract_sign": ("float kk = rel * cosi - cost;", "float kk = rel * cosi + cost;",
                     "tests/test_oracle_scatter.py::test_ball_lens_paraxial_focus"),
    # the differentiable renderer of Eq. 9
    "dp_interior_hit_motion": ("float dtj = nj / dn;", "float dtj = -nj / dn;",
                               "tests/test_oracle_eq9.py::test_interior_term_matches_central_differences"),
    "dp_silhouette_speed_sign": ("vn[0] = (2.0f * rho * n.x) / gn;", "vn[0] = (-2.0f * rho * n.x) / gn;",
                                 "tests/test_oracle_eq9.py::test_silhouette_term_matches_coverage_differences"),
    "dp_silhouette_length": ("float dx = vdot(jx, dp), dy = vdot(jy, dp);",
                             "float dx = vdot(jx, dp), dy = 0.0f * vdot(jy, dp);",
                             "tests/test_oracle_eq9.py::test_silhouette_term_matches_coverage_differences"),
    "dp_shadow_speed": ("vn[1] = (2.0f * ms.y) / gn;", "vn[1] = (ms.y) / gn;",
                        "tests/test_oracle_eq9.py::test_shadow_term_matches_lit_radiance_differences"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pin_catches_mutant(name, tmp_path):
    from oracle import build as OB
    old, new, pin = MUTANTS[name]
    src = open(ORACLE_C).read()
    assert src.count(old) == 1, f"mutation site of {name} not found once"
    mutant_c = tmp_path / "oracle_mutant.c"
    mutant_c.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", *OB.FLAGS, "-I", os.path.join(ROOT, "oracle"), "-o", str(lib),
                    str(mutant_c), "-lm"], check=True)
    env = dict(os.environ, PRDPT_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        pin], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, f"pin {pin} did not fail on mutant {name}:\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout


def test_host_tuned_build_is_bit_identical(tmp_path):
    # the benchmark times a -march=native build; its results must be the
    # tests' bit for bit
    from oracle import build as OB
    lib = OB.build(native=True, out=str(tmp_path / "liboracle_native.so"))
    probe = (
        "import hashlib, numpy as np\n"
        "from oracle import oracle as O\n"
        "from paper_2211_17263_amd import scenes as S\n"
        "pr = S.caustic_problem(seed=3, width=48, height=40, spp=2, n_occluders=3000)\n"
        "osc = O.OracleScene(pr['scene'])\n"
        "ref = osc.reference(pr['theta_ref'], seed=1)\n"
        "r = osc.grad_estimate(ref, pr['theta0'], pr['sigma'], 4, 3, pr['est'])\n"
        "print(hashlib.sha256(r['grad'].tobytes() + r['losses'].tobytes()).hexdigest())\n")
    outs = []
    for path in (None, lib):
        env = dict(os.environ)
        if path:
            env["PRDPT_ORACLE_LIB"] = path
        r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True,
                           text=True, timeout=300, check=True)
        outs.append(r.stdout.strip())
    assert outs[0] == outs[1] and len(outs[0]) == 64
