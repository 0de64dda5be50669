"""Seeded synthetic inputs (graphs, labelled sets, workload recipes) shared by the
oracle tests and the GPU path.  Holds none of the segmentation method's arithmetic."""
from . import configs, graphs  # noqa: F401
