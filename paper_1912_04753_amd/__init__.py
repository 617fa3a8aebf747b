"""Space-time Ripley's K pair-range count on MI355X (gfx950).

The binding to the C-ABI library lives in ``paper_1912_04753_amd.ripk``; it is
loaded on first use so that the seeded input generators in ``workloads`` can
be imported on a machine without the built library.
"""
