"""The kernel build id used to match a committed rocprofv3 traffic profile to
the current kernels: insensitive to comments and layout, sensitive to code."""
from paper_2107_13500_amd import _strip_comments, kernel_sources_sha256


def test_comments_and_layout_do_not_count():
    a = "int f(int x) {  // twice\n    return 2 * x; /* doubled */\n}\n"
    b = "int f(int x) {\n  return 2 * x;\n}  // same code\n"
    assert _strip_comments(a) == _strip_comments(b)


def test_code_counts():
    assert _strip_comments("return 2 * x;") != _strip_comments("return 3 * x;")


def test_comment_markers_inside_literals_are_code():
    assert _strip_comments('s = "a // b"; c = \'/\';') == 's = "a // b"; c = \'/\';'


def test_build_id_is_stable():
    assert kernel_sources_sha256() == kernel_sources_sha256()
    assert len(kernel_sources_sha256()) == 64
