"""Host logic of the profile summaries: the hash that ties stored HBM counters to the kernel sources
ignores comments and layout but not code; pass kinds are read from kernel names."""

import os

from paper_1602_03395_amd import profiling as pr


def _sources():
    out = {}
    for name in pr.KERNEL_SOURCES:
        with open(os.path.join(os.path.dirname(pr.__file__), "csrc", name), encoding="utf-8") as f:
            out[name] = f.read()
    return out


def test_hash_of_files_equals_hash_of_their_text():
    assert pr.kernels_hash() == pr.kernels_hash(_sources())


def test_comment_and_layout_edits_keep_the_hash_and_code_edits_change_it():
    src = _sources()
    base = pr.kernels_hash(src)
    name = "kernels_cfp.hip"
    commented = dict(src)
    commented[name] = "// a new comment line\n\n" + src[name].replace("\n", "  // trailing note\n", 3)
    assert pr.kernels_hash(commented) == base
    reflowed = dict(src)
    snippet = "    const int tid = (int)threadIdx.x;"
    assert snippet in src[name]
    reflowed[name] = src[name].replace(snippet, "    const int tid =\n        (int) threadIdx.x ;")
    assert pr.kernels_hash(reflowed) == base
    edited = dict(src)
    edited[name] = src[name] + "\nstatic int extra_symbol = 1;\n"
    assert pr.kernels_hash(edited) != base


def test_code_lines_drop_comments_and_blank_lines():
    text = "int a = 1;  // one\n\n   \n// only a comment\nint b = 2;\n"
    assert list(pr.code_lines(text)) == ["int a = 1;", "int b = 2;"]


def test_pass_kinds_of_kernel_names():
    assert pr.pass_kind("k_EAW<float,8,true>") == "EA"
    assert pr.pass_kind("k_ER<float,16,true>") == "E"
    assert pr.pass_kind("k_AAR<float,32,2>") == "AA"
    assert pr.pass_kind("k_EHG<float,64,2>") == "EH"
    assert pr.pass_kind("__amd_rocclr_copyBuffer") is None
