"""MI355X-native multipolar Ewald QM/MM coupling (HIP kernels behind a C ABI).

Submodules are imported lazily so that the seeded input generators
(`workloads`) can be used without loading the HIP library.
"""
__all__ = ["workloads", "ewald"]
