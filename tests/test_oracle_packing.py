"""Pins of the oracle's several-balls-per-simplex layout ("packed"): the
closed form on an equilateral triangle and a regular tetrahedron, the
tangencies the rule is built from on random simplices, and disjoint balls
strictly inside every cell of jittered meshes (Sec. 3: disjoint balls
strictly inside K; eq. def:porous.density for rho_K)."""

import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import transfer as otr
from paper_1908_05834_amd import inputs

S = geo.PACK_SHRINK


def _one(vertices):
    V = np.asarray(vertices, dtype=np.float64)
    return {"kind": "simplex", "vertices": V, "cells": np.arange(V.shape[0])[None, :],
            "phi": np.ones(1)}


def test_equilateral_triangle_closed_form():
    """Side 1: incentre = centroid, r = 1/(2 sqrt 3), each vertex at 2r from
    the incentre, so t = (2r - r)/(2r + r) = 1/3: corner radius r/3,
    centre at a third of the way to the incentre."""
    V = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, math.sqrt(3.0) / 2.0]])
    c, r, cell = geo.simplex_packed_layout(_one(V))
    assert cell.tolist() == [0, 0, 0, 0]
    r_in = 1.0 / (2.0 * math.sqrt(3.0))
    g = V.mean(axis=0)
    assert np.allclose(c[0], g, atol=1e-15, rtol=0)
    assert math.isclose(r[0], S * r_in, rel_tol=1e-15)
    for i in range(3):
        assert np.allclose(c[1 + i], V[i] + (g - V[i]) / 3.0, atol=1e-15, rtol=0)
        assert math.isclose(r[1 + i], S * r_in / 3.0, rel_tol=1e-14)


def test_regular_tetrahedron_closed_form():
    """Edge sqrt 2 (alternate cube corners): incentre = centroid, r = 3 |K| /
    (4 face area), every vertex at 3r from the incentre, so t = (3r - r) /
    (3r + r) = 1/2."""
    V = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 0.0], [1.0, 0.0, 1.0], [0.0, 1.0, 1.0]])
    c, r, cell = geo.simplex_packed_layout(_one(V))
    assert cell.tolist() == [0] * 5
    g = V.mean(axis=0)
    vol = 1.0 / 3.0
    face = math.sqrt(3.0) / 4.0 * 2.0          # equilateral triangle of side sqrt 2
    r_in = 3.0 * vol / (4.0 * face)
    assert np.allclose(c[0], g, atol=1e-15, rtol=0)
    assert math.isclose(r[0], S * r_in, rel_tol=1e-14)
    assert math.isclose(np.linalg.norm(V[0] - g), 3.0 * r_in, rel_tol=1e-14)
    for i in range(4):
        assert np.allclose(c[1 + i], V[i] + 0.5 * (g - V[i]), atol=1e-15, rtol=0)
        assert math.isclose(r[1 + i], S * r_in / 2.0, rel_tol=1e-14)


def _facet_distance(P, pts):
    """Distances from pts to the hyperplane through the dim points P."""
    if P.shape[1] == 2:
        e = P[1] - P[0]
        n = np.array([-e[1], e[0]])
    else:
        n = np.cross(P[1] - P[0], P[2] - P[0])
    n = n / np.linalg.norm(n)
    return np.abs((pts - P[0]) @ n)


@pytest.mark.parametrize("dim", [2, 3])
def test_tangencies_on_random_simplices(dim):
    """Before the shrink the inscribed ball touches every facet and each
    corner ball touches the facets through its vertex and the inscribed
    ball: checked with an independent facet-distance computation."""
    rng = np.random.default_rng(40 + dim)
    for _ in range(30):
        V = rng.uniform(size=(dim + 1, dim))
        if abs(np.linalg.det(V[1:] - V[0])) < 1e-2:
            continue
        c, r, _ = geo.simplex_packed_layout(_one(V), shrink=1.0)
        rin = r[0]
        for i in range(dim + 1):
            others = [j for j in range(dim + 1) if j != i]
            assert math.isclose(_facet_distance(V[others], c[:1])[0], rin, rel_tol=1e-9)
        if c.shape[0] == 1:
            continue
        for i in range(dim + 1):
            ci, ri = c[1 + i], r[1 + i]
            assert math.isclose(np.linalg.norm(ci - c[0]), rin + ri, rel_tol=1e-9)
            for j in range(dim + 1):
                if j == i:
                    continue
                # the facets through v_i: those opposite the other vertices
                others = [k for k in range(dim + 1) if k != j]
                assert math.isclose(_facet_distance(V[others], ci[None])[0], ri, rel_tol=1e-9)


@pytest.mark.parametrize("name", ["tris", "tets"])
def test_balls_disjoint_and_inside_on_meshes(name):
    mesh = (inputs.triangulated_square(12, 0.15, 3) if name == "tris"
            else inputs.kuhn_tets(4, 0.15, 3))
    dim = mesh["vertices"].shape[1]
    c, r, cell = geo.simplex_packed_layout(mesh)
    nc = mesh["cells"].shape[0]
    counts = np.bincount(cell, minlength=nc)
    assert counts.min() >= 1 and np.mean(counts == dim + 2) > 0.9
    V = mesh["vertices"]
    for K in range(nc):
        idx = np.nonzero(cell == K)[0]
        P = V[mesh["cells"][K]]
        for q in idx:
            for i in range(dim + 1):
                others = [j for j in range(dim + 1) if j != i]
                assert _facet_distance(P[others], c[q][None])[0] > r[q]
        for a in idx:
            for b in idx:
                if a < b:
                    assert np.linalg.norm(c[a] - c[b]) > r[a] + r[b]
    # rho_K |sum of the balls| = |K| (eq. def:porous.density)
    out = otr.build_transfer(mesh, inputs.sample_velocity_grid(
        (12, 12) if dim == 2 else (4, 4, 4), lambda p, t: np.zeros_like(p)), 0.01,
        layout="packed", stop_after="pairs")
    meas = np.bincount(cell, weights=geo.ball_measure(r, dim), minlength=nc)
    assert np.allclose(out["rho"] * meas, out["cell_vol"], rtol=1e-14, atol=0)
