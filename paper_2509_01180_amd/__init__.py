"""MI355X-native ball-harmonic rotational alignment (arXiv 2509.01180).

The compute path is the HIP library libbh.so (C ABI in include/bh.h);
``paper_2509_01180_amd.api`` binds it for torch device tensors.
"""

from ._lib import LIB_PATH, BhError  # noqa: F401


def __getattr__(name):
    # The binding imports torch; load it on first use only.
    if name in ("Plan", "index_size", "index_table", "radial_table", "ball_voxels",
                "dense_xi_size"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
