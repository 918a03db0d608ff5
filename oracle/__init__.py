"""FP64 CPU oracle of the superquadric renderer.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg; never by the product path."""
from .sqr_oracle import *  # noqa: F401,F403
from .sqr_oracle import loss_value  # noqa: F401
from .voxelisation import labels_from, voxel_centres, voxelise  # noqa: F401
from .loss import fused_loss  # noqa: F401
