"""Seeded synthetic inputs for the forest-of-octrees raycaster.

This package builds forests (leaves in space-filling-curve order), per-leaf
coefficient fields and cameras.  It holds none of the rendering arithmetic:
no ray intersection, no segment evaluation and no compositing.  Both the HIP
path and the CPU oracle consume what it produces.
"""

from .scene import (  # noqa: F401
    QMAX,
    Camera,
    Fields,
    Forest,
    Scene,
    config_scene,
    config4_cameras,
    shell_scene,
    shell_map,
    shell_frame,
    shell_params,
    SHELL_R0,
    SHELL_R1,
    morton_keys,
    orthographic_axis_camera,
    perspective_camera,
    random_perspective_camera,
    small_scene,
    uniform_forest,
    adaptive_forest,
    gaussian_sum,
    perturb_fields,
    trilinear_fields_from_gaussians,
    constant_fields,
    constant_variant,
    equilibrium_fields,
    split_shares,
    stack_channels,
)
from .surface import (  # noqa: F401
    gl_nodes,
    ho_geom,
    ho_hexagon_trees,
    ho_random_forest,
    ho_surface_forest,
    ho_tree,
    hexagon_cameras,
    hexagon_corners,
    leaf_corner_points,
    mandelbrot_count,
    mandelbrot_fields,
    mandelbrot_forest,
    patch_point,
    random_quadtree_forest,
    random_surface_fields,
    surface_forest,
)
from .volume import (  # noqa: F401
    bent_map,
    random_quadratic_map,
    vol_geom,
    vol_tree,
    volume_forest,
    volume_scene,
)
