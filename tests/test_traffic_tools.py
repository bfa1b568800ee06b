"""Host-side helpers of the profile summaries (no GPU needed): the kernel-sources hash that ties a
committed counter or trace summary to the code it measured ignores comments, and nothing else."""
from paper_2306_17537_amd import traffic


def test_code_only_drops_comments_and_blank_lines():
    src = "int a = 1;  // one\n\n/* block\n comment */int b = 2;\n   // only a comment\nint c;\n"
    assert traffic._code_only(src) == "int a = 1;\nint b = 2;\nint c;"


def test_comment_edits_keep_the_hash_and_code_edits_change_it():
    base = "template <int L>\n__global__ void k(float* x) {  // scale\n  x[0] *= L;\n}\n"
    reworded = "// a kernel\ntemplate <int L>\n__global__ void k(float* x) {  // times L\n  x[0] *= L;\n}\n"
    changed = base.replace("*= L", "*= 2 * L")
    assert traffic._code_only(base) == traffic._code_only(reworded)
    assert traffic._code_only(base) != traffic._code_only(changed)
    assert len(traffic.sources_hash()) == 16
