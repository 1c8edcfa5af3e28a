"""Planted mistakes in the oracle (on the CPU): each mutant of the C source must
fail at least one pin, showing that the pins can tell a wrong oracle from a
right one.  The mutants are built from a textual edit of the source into a
temporary directory; the committed oracle is never modified."""
from __future__ import annotations

import os
import subprocess
import tempfile

import pytest

import oracle
from tests._pins import PINS

MUTANTS = {
    "drop_face_gate": ("if (!(w[0] > 0.0 && w[1] > 0.0 && w[2] > 0.0)) return INFINITY;", ""),
    "drop_edge_gate": ("if (!(t > lo_t && t < hi_t)) return INFINITY;", ""),
    "bary_operand_swap": ("w[1] = dot(cross(sub(c, p), sub(a, p)), n) / nn;",
                          "w[1] = dot(cross(sub(a, p), sub(c, p)), n) / nn;"),
    "foot_sign": ("d3 p = sub(q, scl(n, dot(sub(q, a), n) / nn));",
                  "d3 p = sub(q, scl(n, dot(sub(a, q), n) / nn));"),
    "dot_dropped_term": ("return a.x * b.x + a.y * b.y + a.z * b.z;", "return a.x * b.x + a.y * b.y;"),
    "edge_wrong_index": ("b = F[3 * f + (s + 1) % 3];", "b = F[3 * f + (s + 1) % 2];"),
    "vertex_loop_short": ("for (int64_t k = 0; k < nv; ++k) {\n            double d = vertex_dist",
                          "for (int64_t k = 0; k + 1 < nv; ++k) {\n            double d = vertex_dist"),
    "edge_t_wrong_denominator": ("double t = dot(sub(q, a), ab) / dot(ab, ab);\n    *t_out = t;",
                                 "double t = dot(sub(q, a), ab) / norm(ab);\n    *t_out = t;"),
    "cross_sign": ("a.z * b.x - a.x * b.z", "a.x * b.z - a.z * b.x"),
    # the acceptance helpers: a near-optimal set that admits too much, a
    # relaxed edge gate with the wrong sign, a point-to-primitive distance
    # that ignores the point
    "near_set_admits_every_face": ("if (off <= tol && norm(sub(q, p)) <= dstar + tol) {", "if (1) {"),
    "near_set_admits_every_edge": ("if (!(t >= -r && t <= 1.0 + r)) continue;\n"
                                   "        if (norm(sub(q, add(a, scl(ab, t)))) <= dstar + tol) {",
                                   "if (1) {"),
    "near_set_face_foot_ignored": ("if (off <= tol && norm(sub(q, p)) <= dstar + tol) {",
                                   "if (norm(sub(q, p)) <= dstar + tol) {"),
    "near_set_edge_gate_sign": ("if (!(t >= -r && t <= 1.0 + r)) continue;", "if (!(t >= r && t <= 1.0 + r)) continue;"),
    "point_to_primitive_zero": ("d3 x = mk(x3[0], x3[1], x3[2]);\n    if (type == O_VERTEX)",
                                "d3 x = mk(x3[0], x3[1], x3[2]);\n    return 0.0 * x.x;\n    if (type == O_VERTEX)"),
    "point_to_primitive_face_plane_only": (
        "d3 c = closest_on_triangle(x, at(V, F[3 * id]), at(V, F[3 * id + 1]), at(V, F[3 * id + 2]));\n"
        "        return norm(sub(x, c));",
        "double w[3];\n        d3 c = face_foot(x, at(V, F[3 * id]), at(V, F[3 * id + 1]), at(V, F[3 * id + 2]), w);\n"
        "        return norm(sub(x, c));"),
}


@pytest.fixture(scope="module")
def src():
    with open(oracle.SRC_PATH) as fh:
        return fh.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, src):
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = src.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "m.c")
        so = os.path.join(d, "libm.so")
        with open(c, "w") as fh:
            fh.write(mutated)
        subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", so, c, "-lm"])
        L = oracle.load(so)
        failed = []
        for pin in PINS:
            try:
                pin(L)
            except (AssertionError, ValueError, IndexError, FloatingPointError):
                failed.append(pin.__name__)
        assert failed, f"mutant {name} passed every pin"
