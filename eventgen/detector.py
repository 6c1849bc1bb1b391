"""Synthetic pixel detector and reconstruction configuration (data only).

This module holds numbers, not arithmetic: the layer geometry of the
synthetic four-barrel / three-disk-per-side pixel detector, the table of
layer pairs the doublet step may connect, the geometric cut values and the
fit's measurement and material constants.  Every literal here is an input
handed unchanged to both the reconstruction library and the CPU oracle, the
way detector conditions are inputs of the paper's Tracks module (Sec. 2).

Units: cm, GeV, tesla.  The curvature of a helix of transverse momentum pT in
the 3.8 T field along +z is kappa = C_KAPPA / pT (1/cm), with
C_KAPPA = 0.299792458 * 3.8 * 0.01 written out as a decimal literal so that
both sides read the same double.
"""

BARREL = 0
DISK = 1

DETECTOR = {
    "name": "pixel-4barrel-3disk",
    "bfield_tesla": 3.8,
    # 0.299792458 GeV/(T m) * 3.8 T * 0.01 m/cm
    "c_kappa": 0.011392113404,
    # id, kind, barrel radius / disk z, barrel |z| half-length / disk r range
    "layers": [
        {"id": 0, "kind": BARREL, "r": 2.9, "zmax": 26.5},
        {"id": 1, "kind": BARREL, "r": 6.8, "zmax": 26.5},
        {"id": 2, "kind": BARREL, "r": 10.9, "zmax": 26.5},
        {"id": 3, "kind": BARREL, "r": 16.0, "zmax": 26.5},
        {"id": 4, "kind": DISK, "z": 29.1, "rmin": 4.5, "rmax": 16.0},
        {"id": 5, "kind": DISK, "z": 36.6, "rmin": 4.5, "rmax": 16.0},
        {"id": 6, "kind": DISK, "z": 44.1, "rmin": 4.5, "rmax": 16.0},
        {"id": 7, "kind": DISK, "z": -29.1, "rmin": 4.5, "rmax": 16.0},
        {"id": 8, "kind": DISK, "z": -36.6, "rmin": 4.5, "rmax": 16.0},
        {"id": 9, "kind": DISK, "z": -44.1, "rmin": 4.5, "rmax": 16.0},
    ],
    # (inner layer, outer layer) pairs a doublet may connect; a DAG of
    # distinct layers covering every consecutive crossing of a prompt
    # track with |eta| < 2.5 and |z_vertex| up to about 15 cm.
    "pairs": [
        (0, 1), (1, 2), (2, 3),
        (0, 4), (1, 4), (2, 4), (4, 5), (5, 6),
        (0, 7), (1, 7), (2, 7), (7, 8), (8, 9),
    ],
    "cuts": {
        # maximum transverse curvature (1/cm): C_KAPPA / 0.25 GeV
        "kmax": 0.045568453616,
        # longitudinal impact window (cm)
        "z0max": 15.0,
        # r-z alignment tolerance of two consecutive cells (dimensionless);
        # keeps 99.9 % of true hit triples of the pu50 workload
        "arz": 0.015,
        # transverse impact of a three-hit circle (cm); keeps about 99 %
        "d0max": 0.1,
    },
    "fit": {
        # r-phi resolution of every hit (cm)
        "sigma_u": 1.0e-3,
        # z resolution of barrel hits (cm)
        "sigma_z": 2.0e-3,
        # r resolution of disk hits (cm)
        "sigma_r": 2.0e-3,
        # material per layer at normal incidence, in radiation lengths
        "x_over_x0": 0.01,
        # curvature floor for the scattering momentum estimate: pT <= 1e4 GeV
        "pt_max": 1.0e4,
    },
    "quality": {
        # output selection: n-tuplets with fewer hits are not output
        # (3: triplets and longer; 4: quadruplets and longer only)
        "min_hits": 3,
        # LOOSE flag: chi2 per degree of freedom at most this in both planes
        "chi2": 5.0,
        # STRICT flag: LOOSE and pT (GeV), |d0| (cm), |z0| (cm) within these
        "pt_min": 0.5,
        "d0_max": 0.05,
        "z0_max": 15.0,
    },
    "vertex": {
        # tracks used: at least this many hits and pT at least pt_min (GeV)
        "min_hits": 4,
        "pt_min": 0.5,
        # density clustering of z0: neighbours within eps (cm), a core has
        # at least min_pts neighbours (itself included)
        "eps": 0.02,
        "min_pts": 6,
    },
}


# Workloads.  Each is a recipe for the generator in eventgen/__init__.py.
WORKLOADS = {
    # tiny barrel-only event: noiseless helices, the oracle finishes at once
    "tiny": dict(
        layers=(0, 1, 2, 3), n_tracks=20, n_vertices=1, vertex_sigma=3.0,
        pt_spectrum="loguniform", pt_lo=1.0, pt_hi=10.0, eta_max=1.2,
        smear=False, scatter=False, efficiency=1.0, noise_fraction=0.0,
        phi_spacing=False),
    # one PU~50-like event
    "pu50": dict(
        layers=tuple(range(10)), n_tracks=1500, n_vertices=10,
        vertex_sigma=5.0, pt_spectrum="powerlaw", pt_lo=0.3, pt_hi=1.0e4,
        eta_max=2.5, smear=True, scatter=True, efficiency=0.97,
        noise_fraction=0.05, phi_spacing=False),
    # one PU~200-like event
    "pu200": dict(
        layers=tuple(range(10)), n_tracks=6000, n_vertices=40,
        vertex_sigma=5.0, pt_spectrum="powerlaw", pt_lo=0.3, pt_hi=1.0e4,
        eta_max=2.5, smear=True, scatter=True, efficiency=0.97,
        noise_fraction=0.15, phi_spacing=False),
}

# Batch and serving mixes draw the track count per event, then use the pu50
# distributions with round(tracks / 150) vertices.
BATCH_TRACKS = (300, 3000)       # uniform integer range, 64-event batches
SERVE_PILEUP = (30, 140)         # uniform integer PU, 30 tracks per PU unit
SERVE_TRACKS_PER_PU = 30
