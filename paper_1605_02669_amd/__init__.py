"""MI355X-native Ant Colony System hot path (arXiv:1605.02669).

``paper_1605_02669_amd.acs`` is the binding of the HIP library ``libacs.so``;
``paper_1605_02669_amd.inputs`` generates seeded synthetic instances.  The
binding is imported on first use so that the input generators stay usable
where the library is not built.
"""

__all__ = ["acs", "inputs"]
