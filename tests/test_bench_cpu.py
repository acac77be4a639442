"""Host arithmetic of bench.py: the batched byte model behind roofline.achieved,
and the source hash that ties committed counter summaries to the kernel code
they were taken on."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_batched_byte_model_of_the_16m_vertex_workload():
    n, nnz = 16_000_000, 128_000_000
    mb = bench.model_bytes(n, nnz, 1000, 128)
    # two CSR passes (row offsets, a 4-byte column and a 1-byte sign per entry)
    assert mb["csr_bytes_per_pass"] == 2 * (4 * (n + 1) + 5 * nnz) == 1_408_000_008
    # a level/parent word written and read per vertex, and the n-bit state
    assert mb["bytes_per_tree"] == 16 * n + n // 8 == 258_000_000
    assert mb["passes"] == 8
    assert mb["bytes_per_launch"] == 8 * 1_408_000_008 + 1000 * 258_000_000 == 269_264_000_064
    assert mb["unbatched_bytes_per_launch"] == 1000 * 1_666_000_008
    # a ragged last pass still reads the CSR once; one tree per pass is unbatched
    assert bench.model_bytes(n, nnz, 129, 128)["passes"] == 2
    one = bench.model_bytes(n, nnz, 5, 1)
    assert one["bytes_per_launch"] == one["unbatched_bytes_per_launch"]


class _Sources(dict):
    """Every sweep source reads as the same small function unless given."""

    def __missing__(self, key):
        return "int f(int x) {\n  return x + 1;\n}\n"


def test_source_hash_ignores_comments_and_spacing_only():
    h0 = bench.kernel_source_sha(_Sources())
    noted = _Sources({"fi_multi.h": "// why\nint f(int x) { /* the next */\n\n return x + 1;  }\n"})
    assert bench.kernel_source_sha(noted) == h0
    changed = _Sources({"fi_multi.h": "int f(int x) {\n  return x + 2;\n}\n"})
    assert bench.kernel_source_sha(changed) != h0
    moved = _Sources({"sweep_multi.hip": "int g;\nint f(int x) {\n  return x + 1;\n}\n"})
    assert bench.kernel_source_sha(moved) != h0
