"""MI355X forest-of-octrees raycasting: visibility, ray segments, sort-free
compositing and the adjoint, as hand-written HIP kernels behind the C ABI of
include/rc.h (librc.so).  This package is the Python binding."""

from ._lib import EXPORTS, LIB_PATH, RcError, lib  # noqa: F401
from .render import (  # noqa: F401
    DeviceCameras,
    DeviceFields,
    DeviceForest,
    DeviceIndex,
    RenderFn,
    Renderer,
    VForest,
    lists_workspace_bytes,
    merge_lists,
    rc_camera_prepare,
    rc_composite,
    rc_composite_lists,
    rc_forest_index,
    rc_merge_lists,
    rc_prune_visible,
    rc_render,
    rc_segments,
    rc_segments_backward,
    render,
)
