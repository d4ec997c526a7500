"""Synthetic channel-flow workloads shaped like the paper's test case (Sec. 3.A).

Plain parameter sets, no arithmetic of the method.  Field names are those of the C ABI
structs (mesh, velocity grid, boundary, options) plus ``kn``; ``bc`` is 0 (periodic) or
1 (channel).
"""

CHANNEL_DEFAULTS = dict(bc=1, inlet_fixed_u=0, p_ratio=2.0, T_in=1.0, T_wall=1.0, U_in=0.0,
                        U_noise=0.0, cfl=0.8, rho0=1.0, T0=1.0, noise=0.01, dt_override=0.0)


def _case(**kw):
    c = dict(CHANNEL_DEFAULTS)
    c.update(kw)
    return c


# Parity case: 40x10 cells on 4x1, 24^2 velocities on [-5,5]^2, Kn 0.1, ratio 2, 100 steps.
C1 = _case(nx=40, ny=10, lx=4.0, ly=1.0, nu=24, nv=24, umax=5.0, vmax=5.0, kn=0.1, seed=1)
C1_STEPS = 100

# Throughput case: 400x100 cells, 40^2 velocities on [-6,6]^2, Kn 0.05, 64M updates/step.
C2 = _case(nx=400, ny=100, lx=4.0, ly=1.0, nu=40, nv=40, umax=6.0, vmax=6.0, kn=0.05, seed=2)
C2_STEPS = 1000

# Wide velocity space: 200x50 cells, 101^2 velocities on [-20,20]^2, Kn 0.5, ratio 1.5,
# inlet U = 0.1 (1 + 0.05 xi_j), no interior noise.
C3 = _case(nx=200, ny=50, lx=4.0, ly=1.0, nu=101, nv=101, umax=20.0, vmax=20.0, kn=0.5,
           p_ratio=1.5, inlet_fixed_u=1, U_in=0.1, U_noise=0.05, noise=0.0, seed=3)
C3_STEPS = 500

# One GPU's share of C2 split over 8 GPUs along x: a 50x100 slab of the same channel (its
# inlet/outlet ghost columns stand where the neighbours' halo columns would be).
C2_SHARE8 = dict(C2, nx=50, lx=0.5)

# Internal degrees of freedom: the same channels for a monatomic gas seen in the plane (one
# internal degree, gamma = 5/3), each velocity carrying G and H.
C1_DOF = dict(C1, dof=1)
C2_DOF = dict(C2, dof=1)

# Shakhov collision model with the Prandtl number of a monatomic gas.
C1_SHAKHOV = dict(C1, prandtl=2.0 / 3.0)
C2_SHAKHOV = dict(C2, prandtl=2.0 / 3.0)

# Precision form: C2 with f stored in FP32.
C4 = dict(C2)
C4_PRECISION = "fp32_store"
C4_STEPS = 1000

# The paper's own channel (L/W = 2, Kn 0.1, p_in/p_out = 1.2/0.8) on its meshes M1-M4 and
# velocity grids 29^2, 49^2, 69^2 (Table 1); the velocity range is our reading.
def paper_mesh(nx, ny, nvel):
    return _case(nx=nx, ny=ny, lx=2.0, ly=1.0, nu=nvel, nv=nvel, umax=5.0, vmax=5.0, kn=0.1,
                 p_ratio=1.5, seed=5)


PAPER_MESHES = [(40, 20), (80, 40), (120, 60), (160, 80)]
PAPER_VGRIDS = [29, 49, 69]


def oracle_kwargs(case):
    """Fields accepted by the oracle's case struct."""
    keys = ("nx", "ny", "lx", "ly", "nu", "nv", "umax", "vmax", "kn", "bc", "inlet_fixed_u",
            "p_ratio", "T_in", "T_wall", "U_in", "U_noise", "cfl", "rho0", "T0", "noise", "seed",
            "dt_override", "dof", "prandtl", "adaptive_dt")
    return {k: case[k] for k in keys if k in case}


def solver_kwargs(case, precision="fp64"):
    c = {k: v for k, v in case.items() if k != "kn"}
    c["precision"] = precision
    return case["kn"], c


def updates(case):
    return case["nx"] * case["ny"] * case["nu"] * case["nv"]
