"""CPU FP64 oracle for the dynamic-ray-tracing (DRT) hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the benchmark's
CPU-baseline leg may import or run anything in this directory; the product path (the
HIP library and its Python binding) never does, and shares no code with it.

The oracle is the plain definition of what DRT computes (Sec. II and III of the paper):
for every time instant t_j = t0 + j*dt it displaces the terminals with the second-order
Taylor formula (eq. Taylor) and every rigid body with constant translational and angular
acceleration (Sec. III-A.1), re-solves the *same* interaction sequence on the displaced
geometry (image method for reflections, Sec. III-A; the unfolded edge closed form for a
diffraction, eq. diff_point; the rigidly carried tile centroid for diffuse scattering,
Sec. III-C), and then evaluates path length, delay, angles, Doppler, the field
coefficient of each ray and the time-variant transfer function H(t, f).  The paper's
local-frame / relative-motion formulation reaches exactly this result; the oracle works
in the global frame, in float64 throughout, vectorised over rays and time with numpy.

Every function that has no independent check in tests/ says "parity unpinned"; none does.
"""
from .kinematics import (terminal_state, rodrigues, body_poses, place_points, rotate,
                         material_velocity)
from .geometry import mirror, reflection_chain, edge_point, direction_angles
from .em import (fresnel_gamma, utd_transition, utd_coefficient, er_norm_directive,
                 er_gain)
from .drt import extrapolate, cfr, run, freq_axis, C0
from .rates import rates, taylor_points
from .profiles import power_profiles, bin_samples, bin_index
from .tracer import trace, path_exists, moved_scene, rebase, with_rays, segments

__all__ = [
    "terminal_state", "rodrigues", "body_poses", "place_points", "rotate",
    "material_velocity", "mirror", "reflection_chain", "edge_point", "direction_angles",
    "fresnel_gamma", "utd_transition", "utd_coefficient", "er_norm_directive", "er_gain",
    "extrapolate", "cfr", "run", "freq_axis", "C0", "rates", "taylor_points",
    "power_profiles", "bin_samples", "bin_index", "trace", "path_exists", "moved_scene", "rebase", "with_rays", "segments",
]
