"""Host logic of the profile summaries: the source hash that decides whether
a committed counter summary still describes a kernel ignores comments and
layout, and nothing else."""

from paper_2101_08878_amd.rocprof_summary import code_of


def test_code_of_drops_comments_and_layout():
    src = ('int a = 1; // a comment\n'
           '/* a block\n   comment */ const char *s = "x // kept"; char c = \'/\';\n'
           '  b   =\n a;')
    assert code_of(src) == 'int a = 1; const char *s = "x // kept"; char c = \'/\'; b = a;'


def test_code_of_sees_code_changes():
    a = "x = y + 1; // same comment"
    assert code_of(a) == code_of("x = y + 1;   /* other */")
    assert code_of(a) != code_of("x = y + 2; // same comment")
    assert code_of('s = "a";') != code_of('s = "b";')
