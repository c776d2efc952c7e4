"""The stage-kernel source hash that ties measured traffic records to the
kernel (paper_2510_05254_amd/traffic.py): comments do not count, code does.
Host logic only; no GPU."""
import os

from paper_2510_05254_amd import traffic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_code_only_drops_comments_and_keeps_literals():
    src = ('int a = 1; // one\n'
           '/* block\n   comment */ int b = 2;\n'
           '\n'
           'const char *s = "// not a comment /* nor this */";\n'
           "char c = '/'; char q = '\\''; // tail\n"
           'static_assert(true, "quote \\" inside");   \n')
    got = traffic.code_only(src)
    assert got.split("\n") == [
        'int a = 1;',
        ' int b = 2;',
        'const char *s = "// not a comment /* nor this */";',
        "char c = '/'; char q = '\\'';",
        'static_assert(true, "quote \\" inside");',
    ]


def test_kernel_hash_ignores_comment_edits_only():
    text = open(os.path.join(ROOT, traffic.KERNEL_SOURCES[0]), encoding="utf-8").read()
    base = traffic.code_only(text)
    assert traffic.code_only(text.replace("namespace dg {", "// an edited comment\nnamespace dg { /* x */", 1)) == base
    assert traffic.code_only(text.replace("namespace dg {", "namespace dg {\nconstexpr int unused_x = 0;", 1)) != base
