"""The pins catch plausible mistakes: each mutant below is the oracle source
with one mistake planted (a dropped square, a dropped impact term, a
reversed tie-break, a path limit off by one, a wrong sign), built with gcc
into a temporary library and loaded in place of the oracle; at least one
pin must then fail.  Everything runs on the CPU; the real oracle is
untouched."""

import os
import shutil
import subprocess
import tempfile

import pytest

import oracle
from tests import test_oracle as pins
from tests import test_oracle_cleaning as cpins
from tests import test_oracle_rechits as rpins
from tests import test_oracle_vertices as vpins

SRC = os.path.join(os.path.dirname(oracle.__file__), "pxt_oracle.c")

MUTANTS = {
    "score_r_z_term_not_squared": ("return q1 * q1 + q2 * q2;", "return q1 + q2 * q2;"),
    "score_impact_term_not_squared": ("return q1 * q1 + q2 * q2;", "return q1 * q1 + q2;"),
    "score_without_impact_term": ("return q1 * q1 + q2 * q2;", "return q1 * q1;"),
    "tie_break_reversed": ("if (ta[i] != tb[i]) return ta[i] < tb[i] ? -1 : 1;",
                           "if (ta[i] != tb[i]) return ta[i] < tb[i] ? 1 : -1;"),
    "tie_break_missing": ("if (ta[i] != tb[i]) return ta[i] < tb[i] ? -1 : 1;",
                          "if (0) return 0;"),
    "path_limit_one_too_long": ("if (hits + 1 > ORC_MAX_HITS_PER_TUPLE) {",
                                "if (hits + 1 > ORC_MAX_HITS_PER_TUPLE + 1) {"),
    "path_limit_one_too_short": ("if (hits + 1 > ORC_MAX_HITS_PER_TUPLE) {",
                                 "if (hits + 1 >= ORC_MAX_HITS_PER_TUPLE) {"),
    "r_z_cross_sign": ("out[0] = fabs(dra * dzb - dza * drb);",
                       "out[0] = fabs(dra * dzb + dza * drb);"),
    "longer_loses": ("if (na != nb) return na > nb ? -1 : 1;",
                     "if (na != nb) return na > nb ? 1 : -1;"),
}

# the pins a mutant is run against (each takes the detector dictionary)
PINS = [
    cpins.test_score_closed_form_on_a_quadruplet,
    cpins.test_score_closed_form_on_its_triplets,
    cpins.test_cleaning_decided_by_the_impact_term,
    lambda det: cpins.test_exact_tie_goes_to_the_lower_hit_tuple(det, True),
    lambda det: cpins.test_exact_tie_goes_to_the_lower_hit_tuple(det, False),
    cpins.test_longest_path_is_kept,
    cpins.test_longer_tuple_beats_a_lower_score,
    cpins.test_exact_tie_across_roots,
    cpins.test_path_longer_than_eight_hits_is_an_error,
    pins.test_cleaning_prefers_longer_then_lower_score,
    lambda det: pins.test_l1_rz_alignment(det, 0.0160, False),
]


# vertex finding: an exclusive neighbour distance, a core threshold off by
# one, an unweighted mean, a border tie sent to the upper core, a strict pT
# selection, chi2 without the weights
VTX_MUTANTS = {
    "vtx_eps_exclusive": ("if (fabs((double)s[b].z - (double)s[a].z) <= c->eps) ++cnt;",
                          "if (fabs((double)s[b].z - (double)s[a].z) < c->eps) ++cnt;"),
    "vtx_core_off_by_one": ("core[a] = cnt >= c->min_pts;", "core[a] = cnt > c->min_pts;"),
    "vtx_unweighted_mean": ("swz += w * (double)s[a].z;", "swz += (double)s[a].z;"),
    "vtx_border_tie_upper": ("if (bb < 0 || d < bd) {", "if (bb < 0 || d <= bd) {"),
    "vtx_pt_selection_strict": ("fabsf(qopt[i]) <= c->qopt_max", "fabsf(qopt[i]) < c->qopt_max"),
    "vtx_chi2_unweighted": ("chi2 += w * r * r;", "chi2 += r * r;"),
}

# RecHits: the pixel centre offset dropped, u and v pitches swapped, no
# radial projection, the limit off by one, the disk rotation's sign
RH_MUTANTS = {
    "rh_no_pixel_centre": ("SU += q * ((double)pix_u[p] + 0.5);", "SU += q * (double)pix_u[p];"),
    "rh_pitches_swapped": ("const double u = T[6] + T[8] * (SU / Q);",
                           "const double u = T[6] + T[9] * (SU / Q);"),
    "rh_no_projection": ("const double f = r / sqrt(r * r + u * u);", "const double f = 1.0;"),
    "rh_limit_off_by_one": ("if (rank >= max_per_module) continue;",
                            "if (rank > max_per_module) continue;"),
    "rh_disk_rotation_sign": ("gy = (r + u) * s + v * c;", "gy = (r + u) * s - v * c;"),
}

RH_PINS = [
    lambda: rpins.test_barrel_single_pixel_on_the_cylinder(1, 37, 200),
    lambda: rpins.test_disk_single_pixel(4),
    rpins.test_charge_weighted_centroid,
    rpins.test_limit_and_offsets,
]

VTX_PINS = [
    vpins.test_two_groups_closed_form,
    vpins.test_weighted_mean_and_chi2_exact,
    vpins.test_core_threshold,
    vpins.test_neighbour_distance_is_inclusive,
    vpins.test_chain_of_cores_is_one_vertex_and_a_gap_splits,
    vpins.test_border_tie_goes_to_the_lower_vertex,
    vpins.test_nearest_core_wins_a_border,
    vpins.test_selection_boundaries,
]


@pytest.fixture(scope="module")
def workdir():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tempfile.mkdtemp()
    yield d
    shutil.rmtree(d, ignore_errors=True)


def _mutant_lib(workdir, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not unique: %s" % name
    path = os.path.join(workdir, name + ".c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = os.path.join(workdir, name + ".so")
    subprocess.check_call(["gcc", "-O1", "-ffp-contract=off", "-shared", "-fPIC", "-o", so,
                           path, "-lm"])
    oracle.lib()  # the real one built and cached first
    return oracle.load_library(so)


@pytest.mark.parametrize("name", sorted(RH_MUTANTS))
def test_rechits_mutant_is_caught(workdir, name, monkeypatch):
    monkeypatch.setattr(oracle, "_lib", _mutant_lib(workdir, name, *RH_MUTANTS[name]))
    failed = []
    for pin in RH_PINS:
        try:
            pin()
        except (AssertionError, ValueError):
            failed.append(pin)
    assert failed, "no pin fails for mutant %s" % name


@pytest.mark.parametrize("name", sorted(VTX_MUTANTS))
def test_vertex_mutant_is_caught(workdir, name, monkeypatch):
    monkeypatch.setattr(oracle, "_lib", _mutant_lib(workdir, name, *VTX_MUTANTS[name]))
    failed = []
    for pin in VTX_PINS:
        try:
            pin()
        except (AssertionError, ValueError):
            failed.append(pin)
    assert failed, "no pin fails for mutant %s" % name


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(det, workdir, name, monkeypatch):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not unique: %s" % name
    path = os.path.join(workdir, name + ".c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = os.path.join(workdir, name + ".so")
    subprocess.check_call(["gcc", "-O1", "-ffp-contract=off", "-shared", "-fPIC", "-o", so,
                           path, "-lm"])
    oracle.lib()  # the real one built and cached first
    monkeypatch.setattr(oracle, "_lib", oracle.load_library(so))
    failed = []
    for pin in PINS:
        try:
            pin(det)
        except (AssertionError, ValueError):
            failed.append(pin)
    assert failed, "no pin fails for mutant %s" % name
